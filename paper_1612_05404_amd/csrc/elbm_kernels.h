// elbm_kernels.h -- gfx950 kernels of one time step of the entropic lattice
// Boltzmann model for charged leaky-dielectric multiphase fluids
// (Lauricella et al., arXiv:1612.05404).  Every launch covers all boxes of a
// context: one thread per node, 256-node blocks that never straddle a box.
//
// Per step (Sec. II.C):
//   k_density      pull + component densities rho_s and psi_s = 1 - exp(-rho_s)
//   k_gradient     19-point gradient of the liquid density -> unit normal, |grad|^2
//   k_interface    curvature K = -div n, theta, charge weights, block partials
//   k_charge_coef  per-box deterministic reduce -> charge scale and jellium
//   k_charge_rhs   q and the Poisson right-hand side
//   k_sor x 2k     red-black SOR half sweeps
//   (gauge)        zero-mean potential for boxes without Dirichlet nodes
//   k_efield       |E|^2 with E = E_ext - grad phi
//   k_alpha        (second stream, beside the kernels from k_gradient on) pull, FP64 alpha
//                  Newton, Carreau beta -> alpha * beta
//   k_collide      pull again, Shan-Chen + electric force, exact-difference
//                  source, write f*
#pragma once

#include "elbm_device.h"
#include "elbm_mlp.h"

namespace elbm {

// Neighbour mask of every node (the geometry is fixed once a box is set):
// bit p set when r + c_p is a solid node or outside a bounded box.  The
// kernels read it instead of 18 neighbour type bytes.
template <typename Lat, typename T, typename F>
__global__ __launch_bounds__(BLK) void k_neighbour_mask(Ptrs<T, F> a, uint32_t *nbm) {
  Node nd;
  decode(a, nd);
  if (!nd.live) return;
  uint32_t msk = 0u;
#pragma unroll
  for (int p = 1; p < Lat::Q; ++p) {
    const int m = nbr(nd.B, nd.x, nd.y, nd.z, Lat::cx[p], Lat::cy[p], Lat::cz[p]);
    if (m < 0 || (a.type[nd.B.off + m] & 3) == K_SOLID) msk |= 1u << p;
  }
  nbm[nd.g] = msk;
}

// Streaming (left side of Eq. lattice-b) by pulling + densities and the
// Shan-Chen pseudo-potential psi = 1 - exp(-rho) (rho_0 = 1).  Sums run in
// the field type F in the order p = 0..18.  inlet_axis >= 0 (the adaptive
// inlet of the jet set-up, Sec. III.B): NOZZLE fluid nodes also sum their
// momentum along that axis, and every block stores its nodes' momentum and
// mass sums (fixed order) for the per-box mean velocity.
template <typename Lat, typename T, typename F, int C>
__global__ __launch_bounds__(BLK) void k_density(Ptrs<T, F> a, int inlet_axis) {
  Node nd;
  decode(a, nd);
  double acc[2] = {0.0, 0.0};
  if (nd.live) {
    const uint8_t tt = a.type[nd.g];
    const int k = tt & 3;
    const bool noz = inlet_axis >= 0 && (tt & B_NOZZLE) && k == K_FLUID;
    const uint32_t msk = a.nbm[nd.g];  // the source of p is the neighbour in direction opp(p)
    int src[Lat::Q];
    bool bb[Lat::Q];
    src[0] = nd.n;
    bb[0] = false;
#pragma unroll
    for (int p = 1; p < Lat::Q; ++p) {
      src[p] = nbr(nd.B, nd.x, nd.y, nd.z, -Lat::cx[p], -Lat::cy[p], -Lat::cz[p]);
      bb[p] = ((msk >> opp(p)) & 1u) || src[p] < 0;
    }
#pragma unroll
    for (int s = 0; s < C; ++s) {
      F r = F(0);
      double j = 0.0;
      if (k == K_INLET || k == K_OUTLET) {
#pragma unroll
        for (int p = 0; p < Lat::Q; ++p) r += F(a.fa[(int64_t)(s * Lat::Q + p) * a.N + nd.g]);
      } else if (k == K_FLUID && inlet_axis < 0) {  // no nozzle sums (a uniform choice: one plain loop)
#pragma unroll
        for (int p = 0; p < Lat::Q; ++p)
          r += F(bb[p] ? a.fa[(int64_t)(s * Lat::Q + opp(p)) * a.N + nd.g]
                       : a.fa[(int64_t)(s * Lat::Q + p) * a.N + nd.B.off + src[p]]);
      } else if (k == K_FLUID) {
#pragma unroll
        for (int p = 0; p < Lat::Q; ++p) {
          const T v = bb[p] ? a.fa[(int64_t)(s * Lat::Q + opp(p)) * a.N + nd.g]
                            : a.fa[(int64_t)(s * Lat::Q + p) * a.N + nd.B.off + src[p]];
          r += F(v);
          if (noz) {
            const int ca = inlet_axis == 0 ? Lat::cx[p] : inlet_axis == 1 ? Lat::cy[p] : Lat::cz[p];
            if (ca) j += double(ca) * double(v);
          }
        }
      }
      a.rho[(int64_t)s * a.N + nd.g] = r;
      a.psi[nd.g * C + s] = (k == K_SOLID) ? F(0) : -expm1(-r);  // [N][C]: one load per neighbour in k_collide
      if (noz) {
        acc[0] += j;
        acc[1] += double(r);
      }
    }
  }
  if (inlet_axis >= 0) block_sum_store<2>(acc, a.noz_part + (int64_t)nd.blk * 2);
}

// LDS slabs of one field around a 256-node block of the linear mapping (a
// block lies in one box): for each z offset dz of the stencil (-1, 0, +1;
// 0 only on D2Q9) the box nodes with local index in [n0 + dz P - H,
// n0 + dz P + BLK + H), P = nx ny, H = nx + 1, which hold every unwrapped
// lattice neighbour of the block's nodes.  Filled by the whole block with
// coalesced loads, then read in place of the per-direction global loads; a
// neighbour outside its slab (a periodic wrap) is read from memory.  A slot
// holds the value of the node whose index it stands for, so every read is
// that node's value, whichever way the neighbour index was formed.
template <typename F, int NS>
struct FieldSlabs {
  const F *lds;
  int lo, L, P, lmax;  // lo: local index of the first slot of the dz = 0 slab
  __device__ __forceinline__ void fill(F *sm, const F *field, const BoxDev &B, int n0, int lmax_) {
    lds = sm;
    lmax = lmax_;
    P = B.nx * B.ny;
    const int H = B.nx + 1;
    L = BLK + 2 * H;
    lo = n0 - H;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const int base = lo + (k - NS / 2) * P;
      for (int i = threadIdx.x; i < L; i += BLK) {
        const int idx = base + i;
        if (idx >= 0 && idx < B.n) sm[k * lmax + i] = field[B.off + idx];
      }
    }
    __syncthreads();
  }
  // value of local node m >= 0, a neighbour at z offset dz
  __device__ __forceinline__ F get(const F *field, const BoxDev &B, int m, int dz) const {
    const int off = m - (lo + dz * P);
    return (off >= 0 && off < L) ? lds[(dz + NS / 2) * lmax + off] : field[B.off + m];
  }
};

// 19-point isotropic gradient G = (1/c_s^2) sum_p w_p c_p rho_A(r + c_p) (a
// solid or outside neighbour takes the centre value), stored as the unit
// normal n = G/|G| (0 where |G| <= 1e-12) and |G|^2.
// STAGE: neighbours from the LDS slabs (lmax: slab stride, the dynamic LDS
// holds Lat::D == 3 ? 3 : 1 slabs of it).
template <typename Lat, typename T, typename F, bool STAGE>
__global__ __launch_bounds__(BLK) void k_gradient(Ptrs<T, F> a, int lmax) {
  Node nd;
  decode(a, nd);
  field_chain_priority(a.prio);  // after the uniform loads of decode
  FieldSlabs<F, Lat::D == 3 ? 3 : 1> sl;
  if constexpr (STAGE) {
    extern __shared__ __align__(16) unsigned char slab_mem[];
    sl.fill(reinterpret_cast<F *>(slab_mem), a.rho, nd.B, (int)(nd.g - threadIdx.x - nd.B.off), lmax);
  }
  if (!nd.live) return;
  F g0 = F(0), g1 = F(0), g2 = F(0);
  if ((a.type[nd.g] & 3) != K_SOLID) {
    const F c = a.rho[nd.g];
    const uint32_t msk = a.nbm[nd.g];
#pragma unroll
    for (int p = 1; p < Lat::Q; ++p) {
      const int m = nbr(nd.B, nd.x, nd.y, nd.z, Lat::cx[p], Lat::cy[p], Lat::cz[p]);
      F v = c;
      if (m >= 0 && !((msk >> p) & 1u)) v = STAGE ? sl.get(a.rho, nd.B, m, Lat::cz[p]) : a.rho[nd.B.off + m];
      // zero lattice-vector components add nothing: skipped (same sums)
      if (Lat::cx[p]) g0 += F(Lat::w(p) * Lat::cx[p]) * v;
      if (Lat::cy[p]) g1 += F(Lat::w(p) * Lat::cy[p]) * v;
      if (Lat::cz[p]) g2 += F(Lat::w(p) * Lat::cz[p]) * v;
    }
    g0 /= F(CS2);
    g1 /= F(CS2);
    g2 /= F(CS2);
  }
  const F gg = g0 * g0 + g1 * g1 + g2 * g2;
  const F m = sqrt(gg);
  const bool ok = m > F(1e-12);
  a.grad[nd.g] = ok ? g0 / m : F(0);
  a.grad[a.N + nd.g] = ok ? g1 / m : F(0);
  a.grad[2 * a.N + nd.g] = ok ? g2 / m : F(0);
  a.grad[3 * a.N + nd.g] = gg;
}

// Mean curvature K = -div n (Eq. surface-curvature, with the sign that makes a
// convex drop positive; a solid or outside neighbour takes the centre
// normal), smoothed Heaviside theta, the two charge weights of Eqs.
// surface-q2 / surface-q3 and their per-block sums (all nodes, Poisson-unknown
// nodes).
template <typename Lat, typename T, typename F>
__global__ __launch_bounds__(BLK) void k_interface(Ptrs<T, F> a, Model M) {
  Node nd;
  decode(a, nd);
  field_chain_priority(a.prio);  // after the uniform loads of decode
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (nd.live) {
    const uint8_t tt = a.type[nd.g];
    F bulk = F(0), surf = F(0);
    if ((tt & 3) != K_SOLID) {
      const F c0 = a.grad[nd.g], c1 = a.grad[a.N + nd.g], c2 = a.grad[2 * a.N + nd.g];
      const uint32_t msk = a.nbm[nd.g];
      F div = F(0);
#pragma unroll
      for (int p = 1; p < Lat::Q; ++p) {
        const int m = nbr(nd.B, nd.x, nd.y, nd.z, Lat::cx[p], Lat::cy[p], Lat::cz[p]);
        const bool in = m >= 0 && !((msk >> p) & 1u);
        const int64_t gm = nd.B.off + (m >= 0 ? m : nd.n);
        // c_p . n(r + c_p): only the nonzero components of c_p (all +-1) are
        // loaded, 30 gathers per node instead of 54; the products are exact,
        // so the sums equal the full three-term ones
        F s = F(-0.0);  // -0 + x == x for every x: the first add folds away
        if (Lat::cx[p]) s += F(Lat::cx[p]) * (in ? a.grad[gm] : c0);
        if (Lat::cy[p]) s += F(Lat::cy[p]) * (in ? a.grad[a.N + gm] : c1);
        if (Lat::cz[p]) s += F(Lat::cz[p]) * (in ? a.grad[2 * a.N + gm] : c2);
        div += F(Lat::w(p)) * s;
      }
      const F K = -div / F(CS2);
      const F rA = a.rho[nd.g];
      const F theta = F(0.5) * (F(1) + tanh((rA - F(M.rho_th)) / F(M.w_theta)));
      bulk = rA * theta;
      F wK = F(1);
      if (M.curvature) wK += sqrt(sqrt(fmax(K, F(0)) / F(M.K_d)));
      surf = a.grad[3 * a.N + nd.g] * wK;
    }
    a.bulk[nd.g] = bulk;
    a.surf[nd.g] = surf;
    acc[0] = bulk;
    acc[1] = surf;
    if (!(tt & B_DIRICHLET)) {
      acc[2] = bulk;
      acc[3] = surf;
    }
  }
  block_sum_store<4>(acc, a.partials + (int64_t)nd.blk * 4);
}

// One block per box: deterministic fixed-order sum of the box's block
// partials; then the charge scales (conserving: Q/integral, generator: xi)
// and the neutralising background qbar = sum_unknown q / N_unknown.
__global__ __launch_bounds__(BLK) void k_charge_coef(const BoxDev *boxes, const double *partials,
                                                     const double *noz_part, double *scal, Model M, int prio) {
  const BoxDev B = boxes[blockIdx.x];
  field_chain_priority(prio);  // after the uniform box load
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const bool noz = M.inlet_mode > 0;
  // each thread sums the partials of blocks i, i + BLK, i + 2 BLK, ... in that
  // order; the loads of eight of them are issued before their adds (a box of
  // 2^23 nodes has 32768 blocks: one dependent load per add cost ~60 us)
  constexpr int U = 8;
  int i = threadIdx.x;
  for (; i + (U - 1) * BLK < B.nblocks; i += U * BLK) {
    double v[U][4], w[U][2];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t b = B.first_block + i + u * BLK;
#pragma unroll
      for (int k = 0; k < 4; ++k) v[u][k] = partials[b * 4 + k];
      w[u][0] = noz ? noz_part[b * 2] : 0.0;
      w[u][1] = noz ? noz_part[b * 2 + 1] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[k] += v[u][k];
      if (noz) {
        acc[4] += w[u][0];
        acc[5] += w[u][1];
      }
    }
  }
  for (; i < B.nblocks; i += BLK) {
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] += partials[(int64_t)(B.first_block + i) * 4 + k];
    if (noz) {
      acc[4] += noz_part[(int64_t)(B.first_block + i) * 2];
      acc[5] += noz_part[(int64_t)(B.first_block + i) * 2 + 1];
    }
  }
  __shared__ double tot[6];
  block_sum_store<6>(acc, tot);
  __syncthreads();
  if (threadIdx.x == 0) {
    double cb, cs;
    if (M.charge_model == ELBM_CHARGE_CONSERVING) {
      cb = tot[0] > 0.0 ? B.Q_b / tot[0] : 0.0;
      cs = tot[1] > 0.0 ? B.Q_s / tot[1] : 0.0;
    } else {
      cb = M.xi_b;
      cs = M.xi_s;
    }
    double *o = scal + (int64_t)blockIdx.x * NSCAL;
    o[0] = cb;
    o[1] = cs;
    o[2] = B.n_unknown > 0 ? (cb * tot[2] + cs * tot[3]) / (double)B.n_unknown : 0.0;
    o[7] = 0.0;  // this step's Poisson solve has not met its tolerance yet
    // mean velocity inside the nozzle: momentum over mass of the NOZZLE nodes
    o[8] = (M.inlet_mode > 0 && tot[5] > 0.0) ? tot[4] / tot[5] : 0.0;
  }
}

__constant__ int kFace[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};

// q and the right-hand side of sum_faces eps_f (phi_nb - phi) =
// sum_faces eps_f E_ext . e_f - (q - qbar)   (Gauss law with eps = 1 + rho_A).
template <typename T, typename F>
__global__ __launch_bounds__(BLK) void k_charge_rhs(Ptrs<T, F> a) {
  Node nd;
  decode(a, nd);
  field_chain_priority(a.prio);  // after the uniform loads of decode
  if (!nd.live) return;
  const double *sc = a.scal + (int64_t)nd.bb * NSCAL;
  const uint8_t tt = a.type[nd.g];
  F q = F(0);
  if ((tt & 3) != K_SOLID) q = F(sc[0]) * a.bulk[nd.g] + F(sc[1]) * a.surf[nd.g];
  a.q[nd.g] = q;
  F r = -(q - F(sc[2]));
  const F ec = F(1) + a.rho[nd.g];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int m = nbr(nd.B, nd.x, nd.y, nd.z, kFace[f][0], kFace[f][1], kFace[f][2]);
    if (m < 0) continue;
    const F ef = F(0.5) * (ec + (F(1) + a.rho[nd.B.off + m]));
    r += ef * F(nd.B.E[0] * kFace[f][0] + nd.B.E[1] * kFace[f][1] + nd.B.E[2] * kFace[f][2]);
  }
  a.rhs[nd.g] = r;
}

// One red-black SOR half sweep over the nodes of one colour ((x+y+z) & 1).
// Every load is issued before the Dirichlet test (one dependent memory round
// trip less); faces leaving the box are skipped.
template <typename T, typename F>
__global__ __launch_bounds__(BLK) void k_sor(Ptrs<T, F> a, int colour, int skip_converged) {
  Node nd;
  decode(a, nd);
  field_chain_priority(a.prio);  // after the uniform loads of decode
  if (!nd.live) return;
  // a box whose solve met its tolerance at a check keeps its potential
  if (skip_converged && a.scal[(int64_t)nd.bb * NSCAL + 7] != 0.0) return;
  if (((nd.x + nd.y + nd.z) & 1) != colour) return;
  const uint8_t tt = a.type[nd.g];
  const F rc = a.rho[nd.g], pc = a.phi[nd.g], rhs = a.rhs[nd.g];
  F rn[6], pn[6];
  unsigned inside = 0u;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int m = nbr(nd.B, nd.x, nd.y, nd.z, kFace[f][0], kFace[f][1], kFace[f][2]);
    if (m >= 0) inside |= 1u << f;
    const int64_t gm = nd.B.off + (m >= 0 ? m : nd.n);
    rn[f] = a.rho[gm];
    pn[f] = a.phi[gm];
  }
  if (tt & B_DIRICHLET) return;
  const F ec = F(1) + rc;
  F A = F(0), Bs = F(0);
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    if (!((inside >> f) & 1u)) continue;
    const F ef = F(0.5) * (ec + (F(1) + rn[f]));
    A += ef;
    Bs += ef * pn[f];
  }
  const F om = F(nd.B.omega);
  a.phi[nd.g] = (F(1) - om) * pc + om * (Bs - rhs) / A;
}

// The same half sweep with one thread per pair of x-consecutive nodes (every
// box has an even x extent): the thread updates the pair's node of this
// colour, so half the waves run and none idles on the other colour.  Each
// wave's 128 nodes lie in one 256-node block (a box starts at a multiple of
// 256 nodes), so the block and its box record are wave-uniform.  Same
// arithmetic per node as k_sor: bit-identical potentials.
template <typename T, typename F>
__global__ __launch_bounds__(BLK) void k_sor_pair(Ptrs<T, F> a, int colour, int skip_converged) {
  const int pb = logical_block((a.nblocks + 1) >> 1, a.remap);  // 512-node block
  const int blk = __builtin_amdgcn_readfirstlane(2 * pb + (threadIdx.x >> 7));
  field_chain_priority(a.prio);
  if (blk >= a.nblocks) return;
  const int bb = a.block_box[blk];
  const BoxDev B = a.boxes[bb];
  const int64_t g0 = (int64_t)blk * BLK + 2 * (threadIdx.x & 127);
  const int n0 = (int)(g0 - B.off);
  if (n0 >= B.n) return;
  if (skip_converged && a.scal[(int64_t)bb * NSCAL + 7] != 0.0) return;
  const int r = div_extent(n0, B.rnx), z = div_extent(r, B.rny);
  const int x0 = n0 - r * B.nx, y = r - z * B.ny;
  const int sh = ((x0 + y + z) & 1) != colour ? 1 : 0;
  const int x = x0 + sh, n = n0 + sh;
  const int64_t g = g0 + sh;
  const uint8_t tt = a.type[g];
  const F rc = a.rho[g], pc = a.phi[g], rhs = a.rhs[g];
  F rn[6], pn[6];
  unsigned inside = 0u;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int m = nbr(B, x, y, z, kFace[f][0], kFace[f][1], kFace[f][2]);
    if (m >= 0) inside |= 1u << f;
    const int64_t gm = B.off + (m >= 0 ? m : n);
    rn[f] = a.rho[gm];
    pn[f] = a.phi[gm];
  }
  if (tt & B_DIRICHLET) return;
  const F ec = F(1) + rc;
  F A = F(0), Bs = F(0);
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    if (!((inside >> f) & 1u)) continue;
    const F ef = F(0.5) * (ec + (F(1) + rn[f]));
    A += ef;
    Bs += ef * pn[f];
  }
  const F om = F(B.omega);
  a.phi[g] = (F(1) - om) * pc + om * (Bs - rhs) / A;
}

// Poisson residual of every unknown node in FP64,
//   r = sum_faces eps_f (phi_nb - phi) - rhs   (faces leaving the box skipped),
// and the block maxima of |r| and |rhs|.  Boxes whose solve already met its
// tolerance this step are skipped (skip_converged).
template <typename T, typename F>
__global__ __launch_bounds__(BLK) void k_residual(Ptrs<T, F> a, int skip_converged) {
  Node nd;
  decode(a, nd);
  field_chain_priority(a.prio);  // after the uniform loads of decode
  double v[2] = {0.0, 0.0};
  bool on = nd.live && !(skip_converged && a.scal[(int64_t)nd.bb * NSCAL + 7] != 0.0);
  if (on) on = !(a.type[nd.g] & B_DIRICHLET);
  if (on) {
    const double ec = 1.0 + double(a.rho[nd.g]);
    const double pc = double(a.phi[nd.g]);
    double acc = 0.0;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      const int m = nbr(nd.B, nd.x, nd.y, nd.z, kFace[f][0], kFace[f][1], kFace[f][2]);
      if (m < 0) continue;
      const int64_t gm = nd.B.off + m;
      acc += 0.5 * (ec + (1.0 + double(a.rho[gm]))) * (double(a.phi[gm]) - pc);
    }
    const double rhs = double(a.rhs[nd.g]);
    v[0] = fabs(acc - rhs);
    v[1] = fabs(rhs);
  }
  block_max_store<2>(v, a.res_part + (int64_t)nd.blk * 2);
}

// One block per box: the box's residual and scale from the block maxima.
// A check (final == 0) with the residual within sor_tol * max|rhs| marks the
// box's solve as done (later sweeps skip it); the final call records the
// sweeps of a box still running and counts (and, with a tolerance, flags) a
// solve that ends above it.  A box done at a check keeps that check's record.
__global__ __launch_bounds__(BLK) void k_res_box(const BoxDev *boxes, const double *res_part, double *scal,
                                                 unsigned long long *cnt, uint32_t *err, double tol, int done,
                                                 int final, int prio) {
  const BoxDev B = boxes[blockIdx.x];
  field_chain_priority(prio);  // after the uniform box load
  double *o = scal + (int64_t)blockIdx.x * NSCAL;
  if (o[7] != 0.0) return;
  double v[2] = {0.0, 0.0};
  for (int i = threadIdx.x; i < B.nblocks; i += BLK) {
    v[0] = fmax(v[0], res_part[(int64_t)(B.first_block + i) * 2]);
    v[1] = fmax(v[1], res_part[(int64_t)(B.first_block + i) * 2 + 1]);
  }
  __shared__ double tot[2];
  block_max_store<2>(v, tot);
  __syncthreads();
  if (threadIdx.x == 0) {
    o[4] = tot[0];
    o[5] = tot[1];
    const bool ok = tot[0] <= tol * tot[1];
    if (!final) {
      if (tol > 0.0 && ok) {
        o[6] = double(done);
        o[7] = 1.0;
      }
    } else {
      o[6] = double(done);
      if (tol > 0.0 && !ok) {
        atomicAdd(cnt + (int64_t)blockIdx.x * NCNT + 5, 1ull);
        atomicOr(err, ERR_SOR);
      }
    }
  }
}

// Zero-mean gauge of the potential for boxes without Dirichlet nodes.
template <typename T, typename F>
__global__ __launch_bounds__(BLK) void k_phi_partials(Ptrs<T, F> a) {
  Node nd;
  decode(a, nd);
  field_chain_priority(a.prio);  // after the uniform loads of decode
  double acc[1] = {nd.live ? double(a.phi[nd.g]) : 0.0};
  block_sum_store<1>(acc, a.partials + (int64_t)nd.blk * 4);
}

__global__ __launch_bounds__(BLK) void k_phi_mean(const BoxDev *boxes, const double *partials,
                                                  double *scal, int prio) {
  const BoxDev B = boxes[blockIdx.x];
  field_chain_priority(prio);  // after the uniform box load
  double acc[1] = {0.0};
  for (int i = threadIdx.x; i < B.nblocks; i += BLK) acc[0] += partials[(int64_t)(B.first_block + i) * 4];
  __shared__ double tot[1];
  block_sum_store<1>(acc, tot);
  __syncthreads();
  if (threadIdx.x == 0) scal[(int64_t)blockIdx.x * NSCAL + 3] = tot[0] / (double)B.n;
}

template <typename T, typename F>
__global__ __launch_bounds__(BLK) void k_phi_sub(Ptrs<T, F> a) {
  Node nd;
  decode(a, nd);
  field_chain_priority(a.prio);  // after the uniform loads of decode
  if (!nd.live || nd.B.has_dirichlet) return;
  a.phi[nd.g] -= F(a.scal[(int64_t)nd.bb * NSCAL + 3]);
}

// |E|^2 with E = E_ext - grad phi (19-point gradient; an outside neighbour
// takes the centre value, wall nodes carry their fixed potential).
template <typename Lat, typename T, typename F, bool STAGE>
__global__ __launch_bounds__(BLK) void k_efield(Ptrs<T, F> a, int lmax) {
  Node nd;
  decode(a, nd);
  field_chain_priority(a.prio);  // after the uniform loads of decode
  FieldSlabs<F, Lat::D == 3 ? 3 : 1> sl;
  if constexpr (STAGE) {
    extern __shared__ __align__(16) unsigned char slab_mem[];
    sl.fill(reinterpret_cast<F *>(slab_mem), a.phi, nd.B, (int)(nd.g - threadIdx.x - nd.B.off), lmax);
  }
  if (!nd.live) return;
  const F c = a.phi[nd.g];
  F g0 = F(0), g1 = F(0), g2 = F(0);
#pragma unroll
  for (int p = 1; p < Lat::Q; ++p) {
    const int m = nbr(nd.B, nd.x, nd.y, nd.z, Lat::cx[p], Lat::cy[p], Lat::cz[p]);
    const F v = m >= 0 ? (STAGE ? sl.get(a.phi, nd.B, m, Lat::cz[p]) : a.phi[nd.B.off + m]) : c;
    // zero lattice-vector components add nothing: skipped (same sums)
    if (Lat::cx[p]) g0 += F(Lat::w(p) * Lat::cx[p]) * v;
    if (Lat::cy[p]) g1 += F(Lat::w(p) * Lat::cy[p]) * v;
    if (Lat::cz[p]) g2 += F(Lat::w(p) * Lat::cz[p]) * v;
  }
  const F e0 = F(nd.B.E[0]) - g0 / F(CS2), e1 = F(nd.B.E[1]) - g1 / F(CS2), e2 = F(nd.B.E[2]) - g2 / F(CS2);
  a.e2[nd.g] = e0 * e0 + e1 * e1 + e2 * e2;
}

// LDS copy of the network, present only in the learned-starter variant.
template <bool LEARN> struct LearnLds {};
template <> struct LearnLds<true> { MlpShared net; };

// x_p = (f_eq_p - f_p)/f_p of every direction into the wave's LDS scratch,
// with the same expression as the alpha set-up pass (bit-identical).
template <typename Lat, typename T>
__device__ __forceinline__ void refill_x(const T *f, double *xs, double rho, double ux, double uy, double uz) {
  const double uu = ux * ux + uy * uy + uz * uz;
#pragma unroll 4
  for (int p = 0; p < Lat::Q; ++p) {
    const double fp = double(f[p * BLK]);
    xs[p * XSTRIDE] = (feq<Lat, double>(p, rho, ux, uy, uz, uu) - fp) * rcp_nr(fp);
  }
}

// Velocity inlet (the jet set-up of Sec. III.B: Poiseuille velocity at the inlet
// nodes, density that of the liquid): each step an inlet node is reset, per
// component, to f_eq(rho_nb, u_bc), rho_nb the w-weighted mean density of its
// fluid neighbours (rho_in when it has none), or, with the adaptive inlet, to
// f_eq(rho_in, ubar u_bc), ubar the mean velocity measured inside the nozzle
// this step.  Written to the output buffer, which the next step pulls from.
template <typename Lat, typename T, typename F, int C>
__device__ __forceinline__ void inlet_store(const Ptrs<T, F> &a, const Model &M, const Node &nd) {
  if (M.inlet_mode > 0) {
    const double ub = a.scal[(int64_t)nd.bb * NSCAL + 8];
    const double ux = ub * double(a.ubc[nd.g]), uy = ub * double(a.ubc[a.N + nd.g]),
                 uz = ub * double(a.ubc[2 * a.N + nd.g]);
    const double uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int s = 0; s < C; ++s) {
#pragma unroll 1
      for (int p = 0; p < Lat::Q; ++p)
        a.fb[(int64_t)(s * Lat::Q + p) * a.N + nd.g] = T(feq<Lat, double>(p, M.rho_in[s], ux, uy, uz, uu));
    }
    return;
  }
  double sw = 0.0, sr[C];
#pragma unroll
  for (int s = 0; s < C; ++s) sr[s] = 0.0;
#pragma unroll 1
  for (int p = 1; p < Lat::Q; ++p) {
    const int m = nbr(nd.B, nd.x, nd.y, nd.z, Lat::cx[p], Lat::cy[p], Lat::cz[p]);
    if (m < 0 || (a.type[nd.B.off + m] & 3) != K_FLUID) continue;
    sw += Lat::w(p);
#pragma unroll
    for (int s = 0; s < C; ++s) sr[s] += Lat::w(p) * double(a.rho[(int64_t)s * a.N + nd.B.off + m]);
  }
  const double ux = double(a.ubc[nd.g]), uy = double(a.ubc[a.N + nd.g]), uz = double(a.ubc[2 * a.N + nd.g]);
  const double uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
  for (int s = 0; s < C; ++s) {
    const double r = sw > 0.0 ? sr[s] / sw : M.rho_in[s];
#pragma unroll 1
    for (int p = 0; p < Lat::Q; ++p) a.fb[(int64_t)(s * Lat::Q + p) * a.N + nd.g] = T(feq<Lat, double>(p, r, ux, uy, uz, uu));
  }
}

// Carreau viscosity (Eqs. strain2, carreau) of one component from the
// components of its non-equilibrium stress Pi = sum_p (f_p - f_eq_p) c_p c_p,
// in the field precision R; nu0 when the Carreau law is off.
template <typename R>
__device__ __forceinline__ double viscosity(const Model &M, double nflow, double P00, double P11, double P22,
                                            double P01, double P02, double P12, double rho, double al) {
  if (!M.carreau) return M.nu0;
  const R Pn = sym3_norm2<R>(R(P00), R(P11), R(P22), R(P01), R(P02), R(P12));
  const R nf = R(nflow);
  const R gd = shear_rate<R>(Pn, R(rho), R(al), R(M.nu0), R(M.nu_inf), R(M.lam), nf);
  const R lg = R(M.lam) * gd;
  return double(R(M.nu_inf) + (R(M.nu0) - R(M.nu_inf)) * pow1p<R>(lg * lg, R(0.5) * (nf - R(1))));
}

// The collision (Eq. lattice-b) in two kernels.  The entropic alpha (Eq.
// entropic) and the Carreau viscosity depend only on the pulled populations,
// not on the forces, so k_alpha needs nothing of the step's field chain
// (densities, charge, Poisson, E) and runs beside it on a second stream; it
// leaves alpha * beta per node and component.  k_collide then adds the forces
// and writes the post-collision populations.

// k_alpha: for each fluid node and component, pull the 19 populations and
// their FP64 moments, (LEARN) run the learned starter over the wave, solve
// alpha in FP64, evaluate the viscosity, store ab = alpha c_s^2/(2 nu + c_s^2).
// Per-lane work is predicated on `fl` so that the matrix-core section runs on
// whole waves.  With FP32 populations two blocks fit a CU's LDS: the register
// budget is held to two waves per SIMD (matrix accumulators included).
template <typename Lat, typename T, typename F, int C, bool LEARN>
__global__ __launch_bounds__(BLK, sizeof(T) == 4 ? 2 : 1) void k_alpha(Ptrs<T, F> a, Model M, MlpDev W, int record) {
  // thread-private LDS: populations of the current component (column p * BLK
  // + tid) and, per wave, x_p (column p * 64 + lane), whose 9.5 KB also hold
  // the starter's two [64][32] bf16 tiles before the alpha solve
  __shared__ T lds_f[Lat::Q * BLK];
  __shared__ __align__(16) double lds_x[Lat::Q * BLK];
  __shared__ __align__(16) LearnLds<LEARN> learn;
  if constexpr (LEARN) mlp_stage(W, learn.net);
  Node nd;
  if (a.tx) decode_tile(a, nd);
  else decode(a, nd);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  unsigned long long c_fb = 0, c_it = 0, c_col = 0;
  const int k = nd.live ? (a.type[nd.g] & 3) : K_SOLID;
  const bool fl = nd.live && k == K_FLUID;
  int nl[Lat::Q];
  unsigned solid = 0u;
  if (fl) {
    // ---- neighbours: local index, solid-or-outside flag
    nl[0] = nd.n;
    solid = a.nbm[nd.g];
#pragma unroll
    for (int p = 1; p < Lat::Q; ++p) {
      nl[p] = nbr(nd.B, nd.x, nd.y, nd.z, Lat::cx[p], Lat::cy[p], Lat::cz[p]);
      if (nl[p] < 0) solid |= 1u << p;  // outside the box: already in the mask; kept as a guard
    }
  }
  T *f = lds_f + threadIdx.x;
  double *xs = lds_x + wv * (Lat::Q * 64) + lane;
#pragma unroll
  for (int s = 0; s < C; ++s) {
    // ---- pulled populations and their moments.  The moments are summed in
    // FP64 whatever the storage: the equilibrium of the alpha solve must carry
    // exactly the density and momentum of f (sum Delta = 0), or the rounding
    // of an FP32 sum swamps the O(|Delta|^2) entropy balance.
    double dr = 1.0, jx = 0.0, jy = 0.0, jz = 0.0;
    if (fl) {
      dr = 0.0;
#pragma unroll
      for (int p = 0; p < Lat::Q; ++p) {
        const int q = opp(p);  // the source r - c_p is the neighbour in direction opp(p)
        const bool bounce = (p != 0) && ((solid >> q) & 1u);
        const T v = bounce ? a.fa[(int64_t)(s * Lat::Q + q) * a.N + nd.g]
                           : a.fa[(int64_t)(s * Lat::Q + p) * a.N + nd.B.off + nl[q]];
        f[p * BLK] = v;
        const double dv = double(v);
        dr += dv;
        // only the nonzero components (+-dv exactly; a zero term adds +-0)
        if (Lat::cx[p]) jx += double(Lat::cx[p]) * dv;
        if (Lat::cy[p]) jy += double(Lat::cy[p]) * dv;
        if (Lat::cz[p]) jz += double(Lat::cz[p]) * dv;
      }
    }
    // divisions, not one reciprocal: every instantiation (plain, learned)
    // then forms the same velocity, so starters agree on the same state
    const double ux = jx / dr, uy = jy / dr, uz = jz / dr;
    // ---- alpha set-up at the component's own velocity (FP64)
    AlphaSetup st{};
    if (fl) st = alpha_setup<Lat, T>(f, xs, dr, ux, uy, uz, M.alpha_guess, M.rtol);
    double a0 = 2.0;
    if constexpr (LEARN) {
      // ---- learned starter on the matrix cores, for waves holding a node
      // where the series starter was rejected.  Its bf16 tiles overlay the
      // wave's x scratch, which is refilled afterwards.
      const bool want = fl && st.want_learned;
      if (__ballot(want) != 0) {
        float z[MLP_IN];
        double sc = 0.0;
        bool valid = false;
        if (want) valid = features_from_x(xs, z, sc);
        z[Lat::Q] = float(sc);
        wave_sync();
        __bf16 *tile = reinterpret_cast<__bf16 *>(lds_x + wv * (Lat::Q * 64));
        put_features(tile, lane, z, valid);
        const float y = mlp_forward_wave(learn.net, tile, tile + 64 * 32, lane);
        if (valid) a0 = 2.0 + sc * double(y);
        if (fl) refill_x<Lat, T>(f, xs, dr, ux, uy, uz);
      }
    }
    if (fl) {
      // ---- alpha: Newton polish from the starter
      const double uu = ux * ux + uy * uy + uz * uz;
      int its;
      const double al = alpha_newton<Lat, T>(f, xs, st, a0, M.rtol, M.newton_max, its, M.alpha_iter == ELBM_ITER_HALLEY);
      c_col += 1;
      if (its < 0) c_fb += 1; else c_it += (unsigned long long)its;
      // ---- viscosity: Newtonian nu0, or Carreau from the shear-rate root,
      // evaluated in the field precision
      using R = F;
      double nu = M.nu0;
      if (M.carreau) {
        // Pi = sum_p (f_p - f_eq_p) c_p c_p: the equilibrium's second moment is
        // rho (c_s^2 I + u u) exactly for this f_eq over the lattice's own axes
        // (none along z on D2Q9, where every c_z and u_z vanish), so only f is
        // summed
        double P00 = 0, P11 = 0, P22 = 0, P01 = 0, P02 = 0, P12 = 0;
#pragma unroll  // fully: the lattice vectors fold and the LDS reads issue together
        for (int p = 0; p < Lat::Q; ++p) {
          // only the nonzero products c_a c_b = +-1 are summed (+-f exactly;
          // a zero term would add +-0 and leave the sum as it is)
          const double d = double(f[p * BLK]);
          if (Lat::cx[p] * Lat::cx[p]) P00 += d;
          if (Lat::cy[p] * Lat::cy[p]) P11 += d;
          if (Lat::cz[p] * Lat::cz[p]) P22 += d;
          if (Lat::cx[p] * Lat::cy[p]) P01 += double(Lat::cx[p] * Lat::cy[p]) * d;
          if (Lat::cx[p] * Lat::cz[p]) P02 += double(Lat::cx[p] * Lat::cz[p]) * d;
          if (Lat::cy[p] * Lat::cz[p]) P12 += double(Lat::cy[p] * Lat::cz[p]) * d;
        }
        P00 -= dr * (CS2 + ux * ux);
        P11 -= dr * (CS2 + uy * uy);
        if (Lat::D == 3) P22 -= dr * (CS2 + uz * uz);
        P01 -= dr * (ux * uy);
        P02 -= dr * (ux * uz);
        P12 -= dr * (uy * uz);
        const R Pn = sym3_norm2<R>(R(P00), R(P11), R(P22), R(P01), R(P02), R(P12));
        const R nf = R(nd.B.n_flow);
        const R gd = shear_rate<R>(Pn, R(dr), R(al), R(M.nu0), R(M.nu_inf), R(M.lam), nf);
        const R lg = R(M.lam) * gd;
        nu = double(R(M.nu_inf) + (R(M.nu0) - R(M.nu_inf)) * pow1p<R>(lg * lg, R(0.5) * (nf - R(1))));
      }
      a.ab[(int64_t)s * a.N + nd.g] = al * (CS2 / (2.0 * nu + CS2));
      if (record) {
        a.rec_alpha[(int64_t)s * a.N + nd.g] = al;
        a.rec_iters[(int64_t)s * a.N + nd.g] = its;
      }
    } else if (nd.live && record) {
      a.rec_alpha[(int64_t)s * a.N + nd.g] = 0.0;
      a.rec_iters[(int64_t)s * a.N + nd.g] = 0;
    }
  }
  // ---- counters: wave sums, one atomic per wave and counter
  c_fb = wave_sum_u64(c_fb);
  c_it = wave_sum_u64(c_it);
  c_col = wave_sum_u64(c_col);
  if (lane == 0) {
    unsigned long long *cn = a.cnt + (int64_t)nd.bb * NCNT;
    if (c_fb) atomicAdd(cn + 0, c_fb);
    if (c_it) atomicAdd(cn + 1, c_it);
    if (c_col) atomicAdd(cn + 4, c_col);
    if (c_fb && (M.strict & ELBM_STRICT_ALPHA)) atomicOr(a.err, ERR_ALPHA);
  }
}

// k_collide: at fluid nodes the Shan-Chen (Eq. sc) and electric (Eq.
// force_el2) forces, then per component the pulled populations again (the
// same loads and FP64 moments as k_alpha) and the update
//   f* = f + ab (f_eq - f) + f_eq(rho, u + F/rho) - f_eq(rho, u)
// (exact-difference source, Eq. add).  Inlet nodes are reset; the recorded
// half-step velocity is stored on request.
template <typename Lat, typename T, typename F, int C>
__global__ __launch_bounds__(BLK) void k_collide(Ptrs<T, F> a, Model M, int record) {
  Node nd;
  decode(a, nd);
  const int lane = threadIdx.x & 63;
  unsigned long long c_neg = 0, c_nf = 0;
  const int k = nd.live ? (a.type[nd.g] & 3) : K_SOLID;
  const bool fl = nd.live && k == K_FLUID;
  unsigned solid = fl ? a.nbm[nd.g] : 0u;  // neighbour p solid or outside (bit p)
  F acc[C][3], wall[3] = {F(0), F(0), F(0)}, Fel[3] = {F(0), F(0), F(0)}, rt = F(1);
#pragma unroll
  for (int s = 0; s < C; ++s) acc[s][0] = acc[s][1] = acc[s][2] = F(0);
  if (fl) {
    // ---- Shan-Chen (Eq. sc) and electric (Eq. force_el2) forces
    F gp[3] = {F(0), F(0), F(0)}, ge[3] = {F(0), F(0), F(0)};
    const F phic = a.phi[nd.g], e2c = a.e2[nd.g];
#pragma unroll
    for (int p = 1; p < Lat::Q; ++p) {
      const int m = nbr(nd.B, nd.x, nd.y, nd.z, Lat::cx[p], Lat::cy[p], Lat::cz[p]);
      const int64_t gm = nd.B.off + (m >= 0 ? m : nd.n);
      if (m < 0) solid |= 1u << p;  // outside the box: already in the mask; kept as a guard
      // zero lattice-vector components add nothing: skipped (same sums)
      if ((solid >> p) & 1u) {
        if (Lat::cx[p]) wall[0] += F(Lat::w(p) * Lat::cx[p]);
        if (Lat::cy[p]) wall[1] += F(Lat::w(p) * Lat::cy[p]);
        if (Lat::cz[p]) wall[2] += F(Lat::w(p) * Lat::cz[p]);
      } else {
        F ps[C];
#pragma unroll
        for (int t = 0; t < C; ++t) ps[t] = a.psi[gm * C + t];
#pragma unroll
        for (int s = 0; s < C; ++s) {
          F sp = F(0);
#pragma unroll
          for (int t = 0; t < C; ++t) sp += F(M.G[s][t]) * ps[t];
          if (Lat::cx[p]) acc[s][0] += F(Lat::w(p)) * sp * F(Lat::cx[p]);
          if (Lat::cy[p]) acc[s][1] += F(Lat::w(p)) * sp * F(Lat::cy[p]);
          if (Lat::cz[p]) acc[s][2] += F(Lat::w(p)) * sp * F(Lat::cz[p]);
        }
      }
      const F vp = m >= 0 ? a.phi[gm] : phic;
      const F ve = m >= 0 ? a.e2[gm] : e2c;
      if (Lat::cx[p]) gp[0] += F(Lat::w(p) * Lat::cx[p]) * vp;
      if (Lat::cy[p]) gp[1] += F(Lat::w(p) * Lat::cy[p]) * vp;
      if (Lat::cz[p]) gp[2] += F(Lat::w(p) * Lat::cz[p]) * vp;
      if (Lat::cx[p]) ge[0] += F(Lat::w(p) * Lat::cx[p]) * ve;
      if (Lat::cy[p]) ge[1] += F(Lat::w(p) * Lat::cy[p]) * ve;
      if (Lat::cz[p]) ge[2] += F(Lat::w(p) * Lat::cz[p]) * ve;
    }
    const F qn = a.q[nd.g];
    const F rA = a.rho[nd.g];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const F E = F(nd.B.E[d]) - gp[d] / F(CS2);
      Fel[d] = qn * E;
      if (M.electrostriction) Fel[d] += F(0.5) * rA * (ge[d] / F(CS2));
    }
    rt = F(0);
#pragma unroll
    for (int s = 0; s < C; ++s) rt += a.rho[(int64_t)s * a.N + nd.g];
  }
  double mom[3] = {0.0, 0.0, 0.0}, drt = 0.0;
#pragma unroll
  for (int s = 0; s < C; ++s) {
    if (!fl) continue;
    // ---- pulled populations and their FP64 moments (as in k_alpha)
    T f[Lat::Q];
    double dr = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int p = 0; p < Lat::Q; ++p) {
      const int q = opp(p);
      const bool bounce = (p != 0) && ((solid >> q) & 1u);
      const int m = p ? nbr(nd.B, nd.x, nd.y, nd.z, Lat::cx[q], Lat::cy[q], Lat::cz[q]) : nd.n;
      f[p] = bounce ? a.fa[(int64_t)(s * Lat::Q + q) * a.N + nd.g]
                    : a.fa[(int64_t)(s * Lat::Q + p) * a.N + nd.B.off + m];
      const double dv = double(f[p]);
      dr += dv;
      // only the nonzero components (+-dv exactly; a zero term adds +-0)
      if (Lat::cx[p]) jx += double(Lat::cx[p]) * dv;
      if (Lat::cy[p]) jy += double(Lat::cy[p]) * dv;
      if (Lat::cz[p]) jz += double(Lat::cz[p]) * dv;
    }
    const double ird = rcp_nr(dr);  // one reciprocal for the three components
    const double ux = jx * ird, uy = jy * ird, uz = jz * ird;
    const double uu = ux * ux + uy * uy + uz * uz;
    drt += dr;
    const F ps = a.psi[nd.g * C + s];
    const F frac = a.rho[(int64_t)s * a.N + nd.g] / rt;
    F gw = F(0);  // wall neighbours carry the node's own psi (Eq. sc, wall sum)
#pragma unroll
    for (int t = 0; t < C; ++t) gw += F(M.Gw[s][t]) * a.psi[nd.g * C + t];
    F Fs[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) Fs[d] = -ps * acc[s][d] - ps * gw * wall[d] + frac * Fel[d];
    mom[0] += jx + 0.5 * double(Fs[0]);
    mom[1] += jy + 0.5 * double(Fs[1]);
    mom[2] += jz + 0.5 * double(Fs[2]);
    const double ab = a.ab[(int64_t)s * a.N + nd.g];
    // ---- exact-difference source (Eq. add): with v = u + F/rho,
    // f_eq(v) - f_eq(u) = w rho [3 c.du + 4.5 (c.du)(c.(u+v)) - 1.5 du.(u+v)]
    const double dx_ = double(Fs[0]) * ird, dy_ = double(Fs[1]) * ird, dz_ = double(Fs[2]) * ird;
    const double sx = 2.0 * ux + dx_, sy = 2.0 * uy + dy_, sz = 2.0 * uz + dz_;
    const double ds = dx_ * sx + dy_ * sy + dz_ * sz;
#pragma unroll
    for (int p = 0; p < Lat::Q; ++p) {
      const double fe = feq<Lat, double>(p, dr, ux, uy, uz, uu);
      // c.d and c.s over the nonzero components only (c_a = +-1: the same
      // sums without the zero terms)
      const double cd = cdot<double>(Lat::cx[p], Lat::cy[p], Lat::cz[p], dx_, dy_, dz_);
      const double cs = cdot<double>(Lat::cx[p], Lat::cy[p], Lat::cz[p], sx, sy, sz);
      const double src = Lat::w(p) * dr * (3.0 * cd + 4.5 * (cd * cs) - 1.5 * ds);
      const double fp = double(f[p]);
      const double v = fp + ab * (fe - fp) + src;
      const T tv = T(v);
      if (!isfinite(tv)) c_nf += 1;
      else if (tv < T(0)) c_neg += 1;
      a.fb[(int64_t)(s * Lat::Q + p) * a.N + nd.g] = tv;
    }
  }
  if (fl && record) {
    a.rec_u[nd.g] = F(mom[0] / drt);
    a.rec_u[a.N + nd.g] = F(mom[1] / drt);
    a.rec_u[2 * a.N + nd.g] = F(mom[2] / drt);
  } else if (nd.live && record) {
    // boundary and wall nodes: recorded velocity sum j / sum rho of their populations
    double r = 0.0, m0 = 0.0, m1 = 0.0, m2 = 0.0;
    if (k != K_SOLID) {
#pragma unroll
      for (int s = 0; s < C; ++s)
#pragma unroll
        for (int p = 0; p < Lat::Q; ++p) {
          const double v = double(a.fa[(int64_t)(s * Lat::Q + p) * a.N + nd.g]);
          r += v;
          m0 += double(Lat::cx[p]) * v;
          m1 += double(Lat::cy[p]) * v;
          m2 += double(Lat::cz[p]) * v;
        }
    }
    a.rec_u[nd.g] = r > 0.0 ? F(m0 / r) : F(0);
    a.rec_u[a.N + nd.g] = r > 0.0 ? F(m1 / r) : F(0);
    a.rec_u[2 * a.N + nd.g] = r > 0.0 ? F(m2 / r) : F(0);
  }
  if (nd.live && k == K_INLET) inlet_store<Lat, T, F, C>(a, M, nd);
  // ---- recorded steps: the electric force summed per block (fixed order)
  if (record) {
    double fe[3] = {double(Fel[0]), double(Fel[1]), double(Fel[2])};
    block_sum_store<3>(fe, a.fel_part + (int64_t)nd.blk * 3);
  }
  // ---- counters: wave sums, one atomic per wave and counter
  c_neg = wave_sum_u64(c_neg);
  c_nf = wave_sum_u64(c_nf);
  if (lane == 0) {
    unsigned long long *cn = a.cnt + (int64_t)nd.bb * NCNT;
    if (c_neg) {
      atomicAdd(cn + 2, c_neg);
      if (M.strict & ELBM_STRICT_NEGPOP) atomicOr(a.err, ERR_NEGPOP);
    }
    if (c_nf) {
      atomicAdd(cn + 3, c_nf);
      atomicOr(a.err, ERR_NONFINITE);
    }
  }
}

// Training samples of the learned starter from the current state of one box:
// for every fluid node and component, the starter input (z [19], s), the
// target (alpha* - 2)/s with alpha* the plain Newton root from 2, the scale s
// and a flag: 0 no features or the plain solve fell back, 1 a valid sample,
// 2 a valid sample where the series starter is rejected (the nodes the
// learned starter serves).  Outputs are indexed s * N_box + n.
template <typename T, typename F, int C>
__global__ __launch_bounds__(BLK) void k_alpha_samples(Ptrs<T, F> a, Model M, int box, float *feat,
                                                       float *target, float *scale, int32_t *valid) {
  __shared__ T lds_f[NQ * BLK];
  __shared__ double lds_x[NQ * BLK];
  Node nd;
  decode(a, nd);
  if (nd.bb != box || !nd.live) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const bool fl = (a.type[nd.g] & 3) == K_FLUID;
  T *f = lds_f + threadIdx.x;
  double *xs = lds_x + wv * (NQ * 64) + lane;
#pragma unroll
  for (int s = 0; s < C; ++s) {
    const int64_t o = (int64_t)s * nd.B.n + nd.n;
    bool ok = false, learned = false;
    float z[NQ];
    double sc = 0.0, al = 2.0;
    if (fl) {
      double dr = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
      for (int p = 0; p < NQ; ++p) {
        const int q = opp(p);
        const int m = p == 0 ? nd.n : nbr(nd.B, nd.x, nd.y, nd.z, kCx[q], kCy[q], kCz[q]);
        const bool bounce = (p != 0) && (m < 0 || (a.type[nd.B.off + m] & 3) == K_SOLID);
        const T v = bounce ? a.fa[(int64_t)(s * NQ + q) * a.N + nd.g]
                           : a.fa[(int64_t)(s * NQ + p) * a.N + nd.B.off + m];
        f[p * BLK] = v;
        const double dv = double(v);
        dr += dv;
        jx += double(kCx[p]) * dv;
        jy += double(kCy[p]) * dv;
        jz += double(kCz[p]) * dv;
      }
      const double ux = jx / dr, uy = jy / dr, uz = jz / dr;
      learned = alpha_setup<D3Q19, T>(f, xs, dr, ux, uy, uz, ELBM_GUESS_MLP, M.rtol).want_learned;
      ok = features_from_x(xs, z, sc);
      const AlphaSetup plain = alpha_setup<D3Q19, T>(f, xs, dr, ux, uy, uz, ELBM_GUESS_STANDARD, M.rtol);
      int its;  // the target: Newton from 2
      al = alpha_newton<D3Q19, T>(f, xs, plain, 2.0, M.rtol, M.newton_max, its);
      ok = ok && its >= 0;
    }
#pragma unroll
    for (int p = 0; p < NQ; ++p) feat[o * MLP_IN + p] = ok ? z[p] : 0.0f;
    feat[o * MLP_IN + NQ] = ok ? float(sc) : 0.0f;
    target[o] = ok ? float((al - 2.0) / sc) : 0.0f;
    scale[o] = ok ? float(sc) : 0.0f;
    valid[o] = ok ? (learned ? 2 : 1) : 0;
  }
}

// ------------------------------------------------------ init / transfer
// Initial populations of direction p of component s for one box.  Staged
// host planes are `ps` doubles apart (the largest box size).
template <typename Lat, typename T, typename F>
__global__ __launch_bounds__(BLK) void k_init_dir(Ptrs<T, F> a, Model M, int box, int s, int p,
                                                  const double *rho0, const double *u0,
                                                  const double *ubc, const double *xi, double amp,
                                                  int64_t ps) {
  const BoxDev B = a.boxes[box];
  const int n = blockIdx.x * BLK + threadIdx.x;
  if (n >= B.n) return;
  const int64_t g = B.off + n;
  const int k = a.type[g] & 3;
  double v = 0.0;
  if (k == K_FLUID) {
    const double ux = u0[n], uy = u0[ps + n], uz = u0[2 * ps + n];
    v = feq<Lat, double>(p, rho0[s * ps + n], ux, uy, uz, ux * ux + uy * uy + uz * uz);
    if (xi) v = v * (1.0 + amp * xi[n]);
  } else if (k == K_INLET) {
    // an adaptive inlet starts from rest (no mean velocity measured yet)
    const bool rest = M.inlet_mode > 0 || !ubc;
    const double ux = rest ? 0.0 : ubc[n], uy = rest ? 0.0 : ubc[ps + n], uz = rest ? 0.0 : ubc[2 * ps + n];
    v = feq<Lat, double>(p, M.rho_in[s], ux, uy, uz, ux * ux + uy * uy + uz * uz);
  } else if (k == K_OUTLET) {
    v = feq<Lat, double>(p, M.rho_out[s], 0.0, 0.0, 0.0, 0.0);
  }
  a.fa[(int64_t)(s * Lat::Q + p) * a.N + g] = T(v);
  a.fb[(int64_t)(s * Lat::Q + p) * a.N + g] = T(v);
}

template <typename X>
__global__ __launch_bounds__(BLK) void k_to_double(const X *src, double *dst, int n) {
  const int i = blockIdx.x * BLK + threadIdx.x;
  if (i < n) dst[i] = double(src[i]);
}
template <typename X>
__global__ __launch_bounds__(BLK) void k_from_double(const double *src, X *dst, X *dst2, int n) {
  const int i = blockIdx.x * BLK + threadIdx.x;
  if (i < n) {
    dst[i] = X(src[i]);
    if (dst2) dst2[i] = X(src[i]);
  }
}

// Partial sums of one box per block, out[blk][9]: mass per component and
// momentum of the current populations, then over the fluid (node,
// component) pairs of the last recorded step the sum and count of alpha,
// -min alpha and max alpha (maxima of non-negative values: alpha > 0).
constexpr int DIAG_W = 9;
template <typename Lat, typename T, typename F, int C>
__global__ __launch_bounds__(BLK) void k_diag(Ptrs<T, F> a, int box, double *out) {
  const BoxDev B = a.boxes[box];
  const int n = blockIdx.x * BLK + threadIdx.x;
  double v[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double mm[2] = {-INFINITY, -INFINITY};
  if (n < B.n) {
    const int64_t g = B.off + n;
#pragma unroll
    for (int s = 0; s < C; ++s)
#pragma unroll
      for (int p = 0; p < Lat::Q; ++p) {
        const double f = double(a.fa[(int64_t)(s * Lat::Q + p) * a.N + g]);
        v[s] += f;
        v[2] += Lat::cx[p] * f;
        v[3] += Lat::cy[p] * f;
        v[4] += Lat::cz[p] * f;
      }
    if ((a.type[g] & 3) == K_FLUID)
#pragma unroll
      for (int s = 0; s < C; ++s) {
        const double al = a.rec_alpha[(int64_t)s * a.N + g];
        v[5] += al;
        v[6] += 1.0;
        mm[0] = fmax(mm[0], -al);
        mm[1] = fmax(mm[1], al);
      }
  }
  block_sum_store<7>(v, out + (int64_t)blockIdx.x * DIAG_W);
  __syncthreads();
  block_max_store<2>(mm, out + (int64_t)blockIdx.x * DIAG_W + 7);
}

}  // namespace elbm
