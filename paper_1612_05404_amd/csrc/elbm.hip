// elbm.hip -- gfx950 kernels and C ABI for the per-time-step update of the
// entropic lattice Boltzmann model for charged leaky-dielectric multiphase
// fluids (Lauricella et al., arXiv:1612.05404).  The ABI is declared and
// documented in include/elbm.h.
//
// Data layout in HBM (one arena owned by the caller):
//   all boxes of a context are concatenated node-wise; every box starts at a
//   multiple of 256 nodes (padding nodes are never touched), so a 256-thread
//   block always lies inside one box.  Every field is structure-of-arrays
//   with one plane of Ntot nodes per component / direction / vector axis:
//   f[(s*19 + p)*Ntot + g], x fastest inside a box.  Populations are double
//   buffered (pull from A, write B, swap).
//
// Per step (Sec. II.C), all boxes in each launch:
//   k_density      pull + component densities rho_s and psi_s = 1 - exp(-rho_s)
//   k_gradient     19-point gradient of the liquid density
//   k_interface    curvature K = -div n, theta, charge weights, block partials
//   k_charge_coef  per-box deterministic reduce -> charge scale and jellium
//   k_charge_rhs   q and the Poisson right-hand side
//   k_sor x 2k     red-black SOR half sweeps
//   (gauge)        zero-mean potential for boxes without Dirichlet nodes
//   k_efield       |E|^2 with E = E_ext - grad phi
//   k_collide      pull again, Shan-Chen + electric force, FP64 alpha Newton,
//                  Carreau beta, exact-difference source, write f*
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

#include "elbm.h"

namespace {

constexpr int NQ = 19;
constexpr int BLK = 256;
constexpr int K_FLUID = 0, K_SOLID = 1, K_INLET = 2, K_OUTLET = 3, B_DIRICHLET = 4;

// D3Q19 velocity set (order documented in elbm.h).
constexpr int kCx[NQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int kCy[NQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int kCz[NQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

__host__ __device__ constexpr double wgt(int p) {
  return p == 0 ? 1.0 / 3.0 : (p < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
}
__host__ __device__ constexpr int opp(int p) { return p == 0 ? 0 : ((p & 1) ? p + 1 : p - 1); }

constexpr double CS2 = 1.0 / 3.0;

struct BoxDev {
  int64_t off;          // first arena node of the box
  int32_t nx, ny, nz, n;
  int32_t per[3];
  int32_t has_dirichlet;
  int32_t first_block, nblocks, n_unknown, pad;
  double E[3];
  double Q_b, Q_s, n_flow, omega;
};

struct Model {
  int32_t C, carreau, curvature, electrostriction, charge_model, newton_max;
  double G[2][2], Gw, nu0, nu_inf, lam, K_d, rho_th, w_theta, xi_b, xi_s, rtol;
  double rho_in[2], rho_out[2];
};

// scalars per box: [0] charge scale of the bulk part, [1] of the surface
// part, [2] neutralising charge qbar, [3] mean potential
constexpr int NSCAL = 8;
// counters per box: fallbacks, Newton updates, negative f, non-finite f, collisions
constexpr int NCNT = 8;

template <typename T>
struct Ptrs {
  T *fa, *fb;           // populations: read fa, write fb
  T *rho, *psi, *grad, *bulk, *surf, *q, *phi, *rhs, *e2;
  T *rec_u;
  double *rec_alpha;
  int32_t *rec_iters;
  uint8_t *type;
  const BoxDev *boxes;
  const int32_t *block_box;
  double *partials;     // [nblocks][4]
  double *scal;         // [nboxes][NSCAL]
  unsigned long long *cnt;  // [nboxes][NCNT]
  uint32_t *err;
  int64_t N;            // arena nodes (plane stride)
};

// ------------------------------------------------------------ node decode
struct Node {
  BoxDev B;
  int bb;
  int64_t g;
  int n, x, y, z;
  bool live;
};

__device__ __forceinline__ void decode(const BoxDev *boxes, const int32_t *block_box, Node &nd) {
  nd.bb = block_box[blockIdx.x];
  nd.B = boxes[nd.bb];
  nd.g = (int64_t)blockIdx.x * BLK + threadIdx.x;
  nd.n = (int)(nd.g - nd.B.off);
  nd.live = nd.n < nd.B.n;
  int t = nd.live ? nd.n : 0;
  nd.x = t % nd.B.nx;
  int r = t / nd.B.nx;
  nd.y = r % nd.B.ny;
  nd.z = r / nd.B.ny;
}

// local index of r + (dx,dy,dz), wrapping periodic axes; -1 outside the box
__device__ __forceinline__ int nbr(const BoxDev &B, int x, int y, int z, int dx, int dy, int dz) {
  int xx = x + dx, yy = y + dy, zz = z + dz;
  if (xx < 0 || xx >= B.nx) {
    if (!B.per[0]) return -1;
    xx = xx < 0 ? xx + B.nx : xx - B.nx;
  }
  if (yy < 0 || yy >= B.ny) {
    if (!B.per[1]) return -1;
    yy = yy < 0 ? yy + B.ny : yy - B.ny;
  }
  if (zz < 0 || zz >= B.nz) {
    if (!B.per[2]) return -1;
    zz = zz < 0 ? zz + B.nz : zz - B.nz;
  }
  return xx + B.nx * (yy + B.ny * zz);
}

// --------------------------------------------------------- reductions
template <int K>
__device__ __forceinline__ void block_sum_store(double (&v)[K], double *out) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += __shfl_xor(v[k], off, 64);
  __shared__ double sm[BLK / 64][K];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) sm[wid][k] = v[k];
  __syncthreads();
  if (threadIdx.x < K) {
    double s = sm[0][threadIdx.x];
#pragma unroll
    for (int w = 1; w < BLK / 64; ++w) s += sm[w][threadIdx.x];
    out[threadIdx.x] = s;
  }
}

// -------------------------------------------------------- equilibrium
template <typename R>
__device__ __forceinline__ R feq(int p, R rho, R ux, R uy, R uz, R uu) {
  const R cu = R(kCx[p]) * ux + R(kCy[p]) * uy + R(kCz[p]) * uz;
  return R(wgt(p)) * rho * (R(1) + cu / R(CS2) + (cu * cu - R(CS2) * uu) / (R(2) * R(CS2) * R(CS2)));
}
// f_eq / (w rho) - 1 without cancellation
__device__ __forceinline__ double feq_dev(int p, double ux, double uy, double uz, double uu) {
  const double cu = double(kCx[p]) * ux + double(kCy[p]) * uy + double(kCz[p]) * uz;
  return cu / CS2 + (cu * cu - CS2 * uu) / (2.0 * CS2 * CS2);
}

// phi(y) = (1+y) ln(1+y) - y, cancellation-free: Taylor series
// sum_{k>=2} (-1)^k y^k / (k(k-1)) through k = 15 for |y| < 1/16 (first
// dropped term below 2e-19 relative), the closed form elsewhere.
__device__ __forceinline__ double phi_fn(double y) {
  if (fabs(y) < 0.0625) {
    double s = -1.0 / 210.0;
    s = fma(s, y, 1.0 / 182.0);
    s = fma(s, y, -1.0 / 156.0);
    s = fma(s, y, 1.0 / 132.0);
    s = fma(s, y, -1.0 / 110.0);
    s = fma(s, y, 1.0 / 90.0);
    s = fma(s, y, -1.0 / 72.0);
    s = fma(s, y, 1.0 / 56.0);
    s = fma(s, y, -1.0 / 42.0);
    s = fma(s, y, 1.0 / 30.0);
    s = fma(s, y, -1.0 / 20.0);
    s = fma(s, y, 1.0 / 12.0);
    s = fma(s, y, -1.0 / 6.0);
    s = fma(s, y, 0.5);
    return s * y * y;
  }
  return (1.0 + y) * log1p(y) - y;
}

// Entropic alpha (Eqs. entropic, H): non-trivial root of
//   g(a) = sum_p f_p phi(a x_p) + a L,  x = (f_eq - f)/f,
//   L = sum_p Delta_p [ln(1 + P_p) - ln(1 + x_p)],  P_p = f_eq_p/(w_p rho) - 1,
// which equals H(f + a Delta) - H(f) exactly (sum Delta = 0).  Newton from a0
// inside the positivity interval (0, a_max); returns the update count or -1
// for the fallback min(2, 0.99 a_max) when no root exists or it is not found.
__device__ double alpha_solve(const double (&f)[NQ], const double (&fe)[NQ], double ux, double uy,
                              double uz, double a0, double rtol, int maxit, int &iters) {
  double x[NQ];
  double xmax = 0.0, amax = INFINITY;
#pragma unroll
  for (int p = 0; p < NQ; ++p) {
    x[p] = (fe[p] - f[p]) / f[p];
    xmax = fmax(xmax, fabs(x[p]));
    if (x[p] < 0.0) amax = fmin(amax, -1.0 / x[p]);
  }
  if (xmax < 1e-12) {
    iters = 0;
    return 2.0;
  }
  const double uu = ux * ux + uy * uy + uz * uz;
  double L = 0.0;
#pragma unroll
  for (int p = 0; p < NQ; ++p)
    L += (fe[p] - f[p]) * (log1p(feq_dev(p, ux, uy, uz, uu)) - log1p(x[p]));
  double a = a0;
  if (!(a > 0.0 && a < amax)) a = 0.5 * fmin(amax, 4.0);
  if (L < 0.0) {
    for (int it = 0; it <= maxit; ++it) {
      double S = 0.0, gp = L;
#pragma unroll
      for (int p = 0; p < NQ; ++p) {
        const double y = a * x[p];
        S += f[p] * phi_fn(y);
        gp += (fe[p] - f[p]) * log1p(y);
      }
      const double g = S + a * L;
      if (fabs(g) <= rtol * S) {
        iters = it;
        return a;
      }
      if (it == maxit) break;
      double an = (gp > 0.0) ? a - g / gp : 2.0 * a;
      if (an >= amax) an = 0.5 * (a + amax);
      if (an <= 0.0) an = 0.5 * a;
      if (fabs(an - a) <= 4.0 * 2.220446049250313e-16 * a) {
        iters = it + 1;
        return an;
      }
      a = an;
    }
  }
  iters = -1;
  return fmin(2.0, 0.99 * amax);
}

// Matrix 2-norm of a symmetric 3x3 (largest |eigenvalue|), cyclic Jacobi.
template <typename R>
__device__ R sym3_norm2(R a00, R a11, R a22, R a01, R a02, R a12) {
  R a[3][3] = {{a00, a01, a02}, {a01, a11, a12}, {a02, a12, a22}};
  for (int sweep = 0; sweep < 12; ++sweep) {
    const R off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    const R diag = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
    if (off <= R(1e-40) * diag || off == R(0)) break;
#pragma unroll
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
      if (a[p][q] == R(0)) continue;
      const R th = (a[q][q] - a[p][p]) / (R(2) * a[p][q]);
      const R t = (th >= R(0) ? R(1) : R(-1)) / (fabs(th) + sqrt(th * th + R(1)));
      const R c = R(1) / sqrt(t * t + R(1)), s = t * c;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const R akp = a[k][p], akq = a[k][q];
        a[k][p] = c * akp - s * akq;
        a[k][q] = s * akp + c * akq;
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const R apk = a[p][k], aqk = a[q][k];
        a[p][k] = c * apk - s * aqk;
        a[q][k] = s * apk + c * aqk;
      }
    }
  }
  return fmax(fabs(a[0][0]), fmax(fabs(a[1][1]), fabs(a[2][2])));
}

// Shear rate of Eq. strain2: root of h(g) = rho (2 nu(g) + c_s^2) g - alpha Pi
// on [0, alpha Pi / (rho (2 nu_inf + c_s^2))], Newton kept in the bracket.
template <typename R>
__device__ R shear_rate(R Pn, R rho, R alpha, R nu0, R ninf, R lam, R n) {
  if (!(Pn > R(0))) return R(0);
  R lo = R(0), hi = alpha * Pn / (rho * (R(2) * ninf + R(CS2)));
  R g = R(0.5) * hi;
  const R tol = sizeof(R) == 8 ? R(1e-15) : R(2e-7);
  for (int it = 0; it < 100; ++it) {
    const R s = R(1) + (lam * g) * (lam * g);
    const R nu = ninf + (nu0 - ninf) * pow(s, R(0.5) * (n - R(1)));
    const R h = rho * (R(2) * nu + R(CS2)) * g - alpha * Pn;
    if (h > R(0)) hi = g; else lo = g;
    const R dh = rho * (R(2) * ninf + R(CS2) +
                        R(2) * (nu0 - ninf) * pow(s, R(0.5) * (n - R(3))) * (R(1) + n * (lam * g) * (lam * g)));
    R gn = g - h / dh;
    if (!(gn > lo && gn < hi)) gn = R(0.5) * (lo + hi);
    if (fabs(gn - g) <= tol * g || hi - lo <= tol * R(0.1) * hi) return gn;
    g = gn;
  }
  return g;
}

// ================================================================ kernels

// Streaming (left side of Eq. lattice-b) by pulling + densities and the
// Shan-Chen pseudo-potential psi = 1 - exp(-rho) (rho_0 = 1).
template <typename T, int C>
__global__ __launch_bounds__(BLK) void k_density(Ptrs<T> a) {
  Node nd;
  decode(a.boxes, a.block_box, nd);
  if (!nd.live) return;
  const int k = a.type[nd.g] & 3;
  int src[NQ];
  bool bb[NQ];
  src[0] = nd.n;
  bb[0] = false;
#pragma unroll
  for (int p = 1; p < NQ; ++p) {
    const int m = nbr(nd.B, nd.x, nd.y, nd.z, -kCx[p], -kCy[p], -kCz[p]);
    bb[p] = (m < 0) || ((a.type[nd.B.off + m] & 3) == K_SOLID);
    src[p] = m;
  }
#pragma unroll
  for (int s = 0; s < C; ++s) {
    T r = T(0);
    if (k == K_INLET || k == K_OUTLET) {
#pragma unroll
      for (int p = 0; p < NQ; ++p) r += a.fa[(int64_t)(s * NQ + p) * a.N + nd.g];
    } else if (k == K_FLUID) {
#pragma unroll
      for (int p = 0; p < NQ; ++p) {
        const T v = bb[p] ? a.fa[(int64_t)(s * NQ + opp(p)) * a.N + nd.g]
                          : a.fa[(int64_t)(s * NQ + p) * a.N + nd.B.off + src[p]];
        r += v;
      }
    }
    a.rho[(int64_t)s * a.N + nd.g] = r;
    a.psi[(int64_t)s * a.N + nd.g] = (k == K_SOLID) ? T(0) : -expm1(-r);
  }
}

// 19-point isotropic gradient (1/c_s^2) sum_p w_p c_p rho_A(r + c_p); a solid
// or outside neighbour takes the centre value.
template <typename T>
__global__ __launch_bounds__(BLK) void k_gradient(Ptrs<T> a) {
  Node nd;
  decode(a.boxes, a.block_box, nd);
  if (!nd.live) return;
  T g0 = T(0), g1 = T(0), g2 = T(0);
  if ((a.type[nd.g] & 3) != K_SOLID) {
    const T c = a.rho[nd.g];
#pragma unroll
    for (int p = 1; p < NQ; ++p) {
      const int m = nbr(nd.B, nd.x, nd.y, nd.z, kCx[p], kCy[p], kCz[p]);
      T v = c;
      if (m >= 0 && (a.type[nd.B.off + m] & 3) != K_SOLID) v = a.rho[nd.B.off + m];
      g0 += T(wgt(p) * kCx[p]) * v;
      g1 += T(wgt(p) * kCy[p]) * v;
      g2 += T(wgt(p) * kCz[p]) * v;
    }
    g0 /= T(CS2);
    g1 /= T(CS2);
    g2 /= T(CS2);
  }
  a.grad[nd.g] = g0;
  a.grad[a.N + nd.g] = g1;
  a.grad[2 * a.N + nd.g] = g2;
}

template <typename T>
__device__ __forceinline__ void unit_normal(const Ptrs<T> &a, int64_t i, T &n0, T &n1, T &n2) {
  const T g0 = a.grad[i], g1 = a.grad[a.N + i], g2 = a.grad[2 * a.N + i];
  const T m = sqrt(g0 * g0 + g1 * g1 + g2 * g2);
  if (m > T(1e-12)) {
    n0 = g0 / m;
    n1 = g1 / m;
    n2 = g2 / m;
  } else {
    n0 = n1 = n2 = T(0);
  }
}

// Mean curvature K = -div n (n = grad rho_A / |grad rho_A|), smoothed
// Heaviside theta, the two charge weights of Eqs. surface-q2 / surface-q3 and
// their per-block sums (all nodes, and Poisson-unknown nodes only).
template <typename T>
__global__ __launch_bounds__(BLK) void k_interface(Ptrs<T> a, Model M) {
  Node nd;
  decode(a.boxes, a.block_box, nd);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (nd.live) {
    const uint8_t tt = a.type[nd.g];
    T bulk = T(0), surf = T(0);
    if ((tt & 3) != K_SOLID) {
      T c0, c1, c2;
      unit_normal(a, nd.g, c0, c1, c2);
      T div = T(0);
#pragma unroll
      for (int p = 1; p < NQ; ++p) {
        const int m = nbr(nd.B, nd.x, nd.y, nd.z, kCx[p], kCy[p], kCz[p]);
        T n0 = c0, n1 = c1, n2 = c2;
        if (m >= 0 && (a.type[nd.B.off + m] & 3) != K_SOLID) unit_normal(a, nd.B.off + m, n0, n1, n2);
        div += T(wgt(p)) * (T(kCx[p]) * n0 + T(kCy[p]) * n1 + T(kCz[p]) * n2);
      }
      const T K = -div / T(CS2);
      const T rA = a.rho[nd.g];
      const T theta = T(0.5) * (T(1) + tanh((rA - T(M.rho_th)) / T(M.w_theta)));
      bulk = rA * theta;
      const T g0 = a.grad[nd.g], g1 = a.grad[a.N + nd.g], g2 = a.grad[2 * a.N + nd.g];
      const T gg = g0 * g0 + g1 * g1 + g2 * g2;
      T wK = T(1);
      if (M.curvature) wK += sqrt(sqrt(fmax(K, T(0)) / T(M.K_d)));
      surf = gg * wK;
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
  block_sum_store<4>(acc, a.partials + (int64_t)blockIdx.x * 4);
}

// One block per box: deterministic fixed-order sum of the box's block
// partials; then the charge scales (conserving: Q/integral, generator: xi)
// and the neutralising background qbar = sum_unknown q / N_unknown.
__global__ __launch_bounds__(BLK) void k_charge_coef(const BoxDev *boxes, const double *partials,
                                                     double *scal, Model M) {
  const BoxDev B = boxes[blockIdx.x];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < B.nblocks; i += BLK)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] += partials[(int64_t)(B.first_block + i) * 4 + k];
  __shared__ double tot[4];
  block_sum_store<4>(acc, tot);
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
    double* o = scal + (int64_t)blockIdx.x * NSCAL;
    o[0] = cb;
    o[1] = cs;
    o[2] = B.n_unknown > 0 ? (cb * tot[2] + cs * tot[3]) / (double)B.n_unknown : 0.0;
  }
}

__constant__ int kFace[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};

// q and the right-hand side of sum_faces eps_f (phi_nb - phi) =
// sum_faces eps_f E_ext . e_f - (q - qbar)   (Gauss law with eps = 1 + rho_A).
template <typename T>
__global__ __launch_bounds__(BLK) void k_charge_rhs(Ptrs<T> a) {
  Node nd;
  decode(a.boxes, a.block_box, nd);
  if (!nd.live) return;
  const double *sc = a.scal + (int64_t)nd.bb * NSCAL;
  const uint8_t tt = a.type[nd.g];
  T q = T(0);
  if ((tt & 3) != K_SOLID) q = T(sc[0]) * a.bulk[nd.g] + T(sc[1]) * a.surf[nd.g];
  a.q[nd.g] = q;
  T r = -(q - T(sc[2]));
  const T ec = T(1) + a.rho[nd.g];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int m = nbr(nd.B, nd.x, nd.y, nd.z, kFace[f][0], kFace[f][1], kFace[f][2]);
    if (m < 0) continue;
    const T ef = T(0.5) * (ec + (T(1) + a.rho[nd.B.off + m]));
    r += ef * T(nd.B.E[0] * kFace[f][0] + nd.B.E[1] * kFace[f][1] + nd.B.E[2] * kFace[f][2]);
  }
  a.rhs[nd.g] = r;
}

// One red-black SOR half sweep over the nodes of one colour ((x+y+z) & 1).
template <typename T>
__global__ __launch_bounds__(BLK) void k_sor(Ptrs<T> a, int colour) {
  Node nd;
  decode(a.boxes, a.block_box, nd);
  if (!nd.live) return;
  if (((nd.x + nd.y + nd.z) & 1) != colour) return;
  if (a.type[nd.g] & B_DIRICHLET) return;
  const T ec = T(1) + a.rho[nd.g];
  T A = T(0), Bs = T(0);
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int m = nbr(nd.B, nd.x, nd.y, nd.z, kFace[f][0], kFace[f][1], kFace[f][2]);
    if (m < 0) continue;
    const int64_t gm = nd.B.off + m;
    const T ef = T(0.5) * (ec + (T(1) + a.rho[gm]));
    A += ef;
    Bs += ef * a.phi[gm];
  }
  const T om = T(nd.B.omega);
  a.phi[nd.g] = (T(1) - om) * a.phi[nd.g] + om * (Bs - a.rhs[nd.g]) / A;
}

// Zero-mean gauge of the potential for boxes without Dirichlet nodes.
template <typename T>
__global__ __launch_bounds__(BLK) void k_phi_partials(Ptrs<T> a) {
  Node nd;
  decode(a.boxes, a.block_box, nd);
  double acc[1] = {nd.live ? double(a.phi[nd.g]) : 0.0};
  block_sum_store<1>(acc, a.partials + (int64_t)blockIdx.x * 4);
}

__global__ __launch_bounds__(BLK) void k_phi_mean(const BoxDev *boxes, const double *partials,
                                                  double *scal) {
  const BoxDev B = boxes[blockIdx.x];
  double acc[1] = {0.0};
  for (int i = threadIdx.x; i < B.nblocks; i += BLK) acc[0] += partials[(int64_t)(B.first_block + i) * 4];
  __shared__ double tot[1];
  block_sum_store<1>(acc, tot);
  __syncthreads();
  if (threadIdx.x == 0) scal[(int64_t)blockIdx.x * NSCAL + 3] = tot[0] / (double)B.n;
}

template <typename T>
__global__ __launch_bounds__(BLK) void k_phi_sub(Ptrs<T> a) {
  Node nd;
  decode(a.boxes, a.block_box, nd);
  if (!nd.live || nd.B.has_dirichlet) return;
  a.phi[nd.g] -= T(a.scal[(int64_t)nd.bb * NSCAL + 3]);
}

// |E|^2 with E = E_ext - grad phi (19-point gradient; an outside neighbour
// takes the centre value, wall nodes carry their fixed potential).
template <typename T>
__global__ __launch_bounds__(BLK) void k_efield(Ptrs<T> a) {
  Node nd;
  decode(a.boxes, a.block_box, nd);
  if (!nd.live) return;
  const T c = a.phi[nd.g];
  T g0 = T(0), g1 = T(0), g2 = T(0);
#pragma unroll
  for (int p = 1; p < NQ; ++p) {
    const int m = nbr(nd.B, nd.x, nd.y, nd.z, kCx[p], kCy[p], kCz[p]);
    const T v = m >= 0 ? a.phi[nd.B.off + m] : c;
    g0 += T(wgt(p) * kCx[p]) * v;
    g1 += T(wgt(p) * kCy[p]) * v;
    g2 += T(wgt(p) * kCz[p]) * v;
  }
  const T e0 = T(nd.B.E[0]) - g0 / T(CS2), e1 = T(nd.B.E[1]) - g1 / T(CS2), e2 = T(nd.B.E[2]) - g2 / T(CS2);
  a.e2[nd.g] = e0 * e0 + e1 * e1 + e2 * e2;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// The collision (Eq. lattice-b) at fluid nodes, with every force term.
template <typename T, int C>
__global__ __launch_bounds__(BLK) void k_collide(Ptrs<T> a, Model M, int record) {
  Node nd;
  decode(a.boxes, a.block_box, nd);
  unsigned long long c_fb = 0, c_it = 0, c_neg = 0, c_nf = 0, c_col = 0;
  const int k = nd.live ? (a.type[nd.g] & 3) : K_SOLID;
  if (nd.live && k == K_FLUID) {
    // ---- neighbours: local index, solid-or-outside flag
    int nl[NQ];
    unsigned solid = 0u;
    nl[0] = nd.n;
#pragma unroll
    for (int p = 1; p < NQ; ++p) {
      nl[p] = nbr(nd.B, nd.x, nd.y, nd.z, kCx[p], kCy[p], kCz[p]);
      if (nl[p] < 0 || (a.type[nd.B.off + nl[p]] & 3) == K_SOLID) solid |= 1u << p;
    }
    // ---- pulled populations and their moments.  The moments are summed in
    // FP64 whatever the storage: the equilibrium of the alpha solve must carry
    // exactly the density and momentum of f (sum Delta = 0), or the rounding
    // of an FP32 sum swamps the O(|Delta|^2) entropy balance.
    T f[C][NQ];
    double rho[C], jx[C], jy[C], jz[C];
    double rt = 0.0;
#pragma unroll
    for (int s = 0; s < C; ++s) {
      rho[s] = 0.0;
      jx[s] = jy[s] = jz[s] = 0.0;
#pragma unroll
      for (int p = 0; p < NQ; ++p) {
        const int q = opp(p);  // the source r - c_p is the neighbour in direction opp(p)
        const bool bounce = (p != 0) && ((solid >> q) & 1u);
        const T v = bounce ? a.fa[(int64_t)(s * NQ + q) * a.N + nd.g]
                           : a.fa[(int64_t)(s * NQ + p) * a.N + nd.B.off + nl[q]];
        f[s][p] = v;
        const double dv = double(v);
        rho[s] += dv;
        jx[s] += double(kCx[p]) * dv;
        jy[s] += double(kCy[p]) * dv;
        jz[s] += double(kCz[p]) * dv;
      }
      rt += rho[s];
    }
    // ---- Shan-Chen (Eq. sc) and electric (Eq. force_el2) forces
    T acc[C][3], wall[3] = {T(0), T(0), T(0)}, gp[3] = {T(0), T(0), T(0)}, ge[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int s = 0; s < C; ++s) acc[s][0] = acc[s][1] = acc[s][2] = T(0);
    const T phic = a.phi[nd.g], e2c = a.e2[nd.g];
#pragma unroll
    for (int p = 1; p < NQ; ++p) {
      const int m = nl[p];
      const int64_t gm = nd.B.off + (m >= 0 ? m : nd.n);
      if ((solid >> p) & 1u) {
        wall[0] += T(wgt(p) * kCx[p]);
        wall[1] += T(wgt(p) * kCy[p]);
        wall[2] += T(wgt(p) * kCz[p]);
      } else {
        T ps[C];
#pragma unroll
        for (int t = 0; t < C; ++t) ps[t] = a.psi[(int64_t)t * a.N + gm];
#pragma unroll
        for (int s = 0; s < C; ++s) {
          T sp = T(0);
#pragma unroll
          for (int t = 0; t < C; ++t) sp += T(M.G[s][t]) * ps[t];
          acc[s][0] += T(wgt(p)) * sp * T(kCx[p]);
          acc[s][1] += T(wgt(p)) * sp * T(kCy[p]);
          acc[s][2] += T(wgt(p)) * sp * T(kCz[p]);
        }
      }
      const T vp = m >= 0 ? a.phi[gm] : phic;
      const T ve = m >= 0 ? a.e2[gm] : e2c;
      gp[0] += T(wgt(p) * kCx[p]) * vp;
      gp[1] += T(wgt(p) * kCy[p]) * vp;
      gp[2] += T(wgt(p) * kCz[p]) * vp;
      ge[0] += T(wgt(p) * kCx[p]) * ve;
      ge[1] += T(wgt(p) * kCy[p]) * ve;
      ge[2] += T(wgt(p) * kCz[p]) * ve;
    }
    const T qn = a.q[nd.g];
    const T rA = a.rho[nd.g];
    T Fel[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const T E = T(nd.B.E[d]) - gp[d] / T(CS2);
      Fel[d] = qn * E;
      if (M.electrostriction) Fel[d] += T(0.5) * rA * (ge[d] / T(CS2));
    }
    double mom[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < C; ++s) {
      const T ps = a.psi[(int64_t)s * a.N + nd.g];
      const T frac = T(rho[s] / rt);
      T F[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) F[d] = -ps * acc[s][d] - T(M.Gw) * ps * ps * wall[d] + frac * Fel[d];
      mom[0] += jx[s] + 0.5 * double(F[0]);
      mom[1] += jy[s] + 0.5 * double(F[1]);
      mom[2] += jz[s] + 0.5 * double(F[2]);
      // ---- equilibrium at the component's own velocity; alpha in FP64
      const double dr = rho[s], dux = jx[s] / dr, duy = jy[s] / dr, duz = jz[s] / dr;
      const double duu = dux * dux + duy * duy + duz * duz;
      double fd[NQ], fe[NQ];
#pragma unroll
      for (int p = 0; p < NQ; ++p) {
        fd[p] = double(f[s][p]);
        fe[p] = feq<double>(p, dr, dux, duy, duz, duu);
      }
      int its;
      const double al = alpha_solve(fd, fe, dux, duy, duz, 2.0, M.rtol, M.newton_max, its);
      c_col += 1;
      if (its < 0) c_fb += 1; else c_it += (unsigned long long)its;
      // ---- viscosity: Newtonian nu0, or Carreau from the shear-rate root
      T nu = T(M.nu0);
      if (M.carreau) {
        T P00 = T(0), P11 = T(0), P22 = T(0), P01 = T(0), P02 = T(0), P12 = T(0);
#pragma unroll
        for (int p = 0; p < NQ; ++p) {
          const T d = T(fd[p] - fe[p]);
          P00 += d * T(kCx[p] * kCx[p]);
          P11 += d * T(kCy[p] * kCy[p]);
          P22 += d * T(kCz[p] * kCz[p]);
          P01 += d * T(kCx[p] * kCy[p]);
          P02 += d * T(kCx[p] * kCz[p]);
          P12 += d * T(kCy[p] * kCz[p]);
        }
        const T Pn = sym3_norm2<T>(P00, P11, P22, P01, P02, P12);
        const T gd = shear_rate<T>(Pn, T(dr), T(al), T(M.nu0), T(M.nu_inf), T(M.lam), T(nd.B.n_flow));
        nu = T(M.nu_inf) + (T(M.nu0) - T(M.nu_inf)) *
                               pow(T(1) + (T(M.lam) * gd) * (T(M.lam) * gd), T(0.5) * (T(nd.B.n_flow) - T(1)));
      }
      const double beta = CS2 / (2.0 * double(nu) + CS2);
      const double ab = al * beta;
      // ---- exact-difference source (Eq. add) and the update
      const double vx = dux + double(F[0]) / dr, vy = duy + double(F[1]) / dr, vz = duz + double(F[2]) / dr;
      const double vv = vx * vx + vy * vy + vz * vz;
#pragma unroll
      for (int p = 0; p < NQ; ++p) {
        const double fe2 = feq<double>(p, dr, vx, vy, vz, vv);
        const double v = fd[p] + ab * (fe[p] - fd[p]) + (fe2 - fe[p]);
        const T tv = T(v);
        if (!isfinite(tv)) c_nf += 1;
        else if (tv < T(0)) c_neg += 1;
        a.fb[(int64_t)(s * NQ + p) * a.N + nd.g] = tv;
      }
      if (record) {
        a.rec_alpha[(int64_t)s * a.N + nd.g] = al;
        a.rec_iters[(int64_t)s * a.N + nd.g] = its;
      }
    }
    if (record) {
      a.rec_u[nd.g] = T(mom[0] / rt);
      a.rec_u[a.N + nd.g] = T(mom[1] / rt);
      a.rec_u[2 * a.N + nd.g] = T(mom[2] / rt);
    }
  } else if (nd.live && record) {
    // boundary and wall nodes: populations stay; recorded velocity sum j / sum rho
    T r = T(0), m0 = T(0), m1 = T(0), m2 = T(0);
    if (k != K_SOLID) {
#pragma unroll
      for (int s = 0; s < C; ++s)
#pragma unroll
        for (int p = 0; p < NQ; ++p) {
          const T v = a.fa[(int64_t)(s * NQ + p) * a.N + nd.g];
          r += v;
          m0 += T(kCx[p]) * v;
          m1 += T(kCy[p]) * v;
          m2 += T(kCz[p]) * v;
        }
    }
    a.rec_u[nd.g] = r > T(0) ? m0 / r : T(0);
    a.rec_u[a.N + nd.g] = r > T(0) ? m1 / r : T(0);
    a.rec_u[2 * a.N + nd.g] = r > T(0) ? m2 / r : T(0);
#pragma unroll
    for (int s = 0; s < C; ++s) {
      a.rec_alpha[(int64_t)s * a.N + nd.g] = 0.0;
      a.rec_iters[(int64_t)s * a.N + nd.g] = 0;
    }
  }
  // ---- counters: wave sums, one atomic per wave and counter
  c_fb = wave_sum_u64(c_fb);
  c_it = wave_sum_u64(c_it);
  c_neg = wave_sum_u64(c_neg);
  c_nf = wave_sum_u64(c_nf);
  c_col = wave_sum_u64(c_col);
  if ((threadIdx.x & 63) == 0) {
    unsigned long long *cn = a.cnt + (int64_t)nd.bb * NCNT;
    if (c_fb) atomicAdd(cn + 0, c_fb);
    if (c_it) atomicAdd(cn + 1, c_it);
    if (c_neg) atomicAdd(cn + 2, c_neg);
    if (c_nf) {
      atomicAdd(cn + 3, c_nf);
      atomicOr(a.err, 1u);
    }
    if (c_col) atomicAdd(cn + 4, c_col);
  }
}

// ------------------------------------------------------ init / transfer
// Initial populations of direction p of component s for one box.
// Staged host planes are `ps` doubles apart (the largest box size).
template <typename T>
__global__ __launch_bounds__(BLK) void k_init_dir(Ptrs<T> a, Model M, int box, int s, int p,
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
    v = feq<double>(p, rho0[s * ps + n], ux, uy, uz, ux * ux + uy * uy + uz * uz);
    if (xi) v = v * (1.0 + amp * xi[n]);
  } else if (k == K_INLET) {
    const double ux = ubc ? ubc[n] : 0.0, uy = ubc ? ubc[ps + n] : 0.0, uz = ubc ? ubc[2 * ps + n] : 0.0;
    v = feq<double>(p, M.rho_in[s], ux, uy, uz, ux * ux + uy * uy + uz * uz);
  } else if (k == K_OUTLET) {
    v = feq<double>(p, M.rho_out[s], 0.0, 0.0, 0.0, 0.0);
  }
  a.fa[(int64_t)(s * NQ + p) * a.N + g] = T(v);
  a.fb[(int64_t)(s * NQ + p) * a.N + g] = T(v);
}

template <typename T>
__global__ __launch_bounds__(BLK) void k_to_double(const T *src, double *dst, int n) {
  const int i = blockIdx.x * BLK + threadIdx.x;
  if (i < n) dst[i] = double(src[i]);
}
template <typename T>
__global__ __launch_bounds__(BLK) void k_from_double(const double *src, T *dst, T *dst2, int n) {
  const int i = blockIdx.x * BLK + threadIdx.x;
  if (i < n) {
    dst[i] = T(src[i]);
    if (dst2) dst2[i] = T(src[i]);
  }
}

// Mass and momentum partial sums of one box's current populations.
template <typename T, int C>
__global__ __launch_bounds__(BLK) void k_diag(Ptrs<T> a, int box, double *out) {
  const BoxDev B = a.boxes[box];
  const int n = blockIdx.x * BLK + threadIdx.x;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  double m1 = 0.0;
  if (n < B.n) {
    const int64_t g = B.off + n;
#pragma unroll
    for (int s = 0; s < C; ++s)
#pragma unroll
      for (int p = 0; p < NQ; ++p) {
        const double v = double(a.fa[(int64_t)(s * NQ + p) * a.N + g]);
        if (s == 0) acc[0] += v; else m1 += v;
        acc[1] += kCx[p] * v;
        acc[2] += kCy[p] * v;
        acc[3] += kCz[p] * v;
      }
  }
  double v5[5] = {acc[0], m1, acc[1], acc[2], acc[3]};
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int k = 0; k < 5; ++k) v5[k] += __shfl_xor(v5[k], off, 64);
  __shared__ double sm[BLK / 64][5];
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < 5; ++k) sm[threadIdx.x >> 6][k] = v5[k];
  __syncthreads();
  if (threadIdx.x < 5) {
    double s = 0.0;
    for (int w = 0; w < BLK / 64; ++w) s += sm[w][threadIdx.x];
    out[(int64_t)blockIdx.x * 5 + threadIdx.x] = s;
  }
}

}  // namespace

// ====================================================================== ABI
struct elbm_ctx {
  elbm_params P;
  std::vector<elbm_box> boxes;
  std::vector<BoxDev> bdev;
  std::vector<int32_t> block_box;
  int64_t Ntot = 0;
  int64_t maxN = 0;
  int nblocks = 0;
  size_t esz = 8;
  // arena offsets (bytes)
  size_t o_fa, o_fb, o_rho, o_psi, o_grad, o_bulk, o_surf, o_q, o_phi, o_rhs, o_e2, o_recu, o_reca,
      o_reci, o_type, o_stage, o_boxes, o_bb, o_part, o_scal, o_cnt, o_err, total;
  char *base = nullptr;
  hipStream_t stream = nullptr;
  bool bound = false;
  bool any_gauge = false;
  int parity = 0;  // which population buffer is current (0: fa region)
  std::string err;
  // device timing: ELBM_NPHASES + 1 events per timed step, recycled
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  double phase_ms[ELBM_NPHASES] = {0, 0, 0, 0, 0};
  int64_t timed_steps = 0;
  ~elbm_ctx() {
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
  }
};

namespace {

elbm_status fail(elbm_ctx *c, elbm_status s, const std::string &msg) {
  if (c) c->err = msg;
  return s;
}

#define HIPCHK(ctx, call)                                                                     \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return fail(ctx, ELBM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

Model make_model(const elbm_params &P) {
  Model M;
  M.C = P.ncomp;
  M.carreau = P.carreau;
  M.curvature = P.curvature;
  M.electrostriction = P.electrostriction;
  M.charge_model = P.charge_model;
  M.newton_max = P.newton_max;
  for (int s = 0; s < 2; ++s)
    for (int t = 0; t < 2; ++t) M.G[s][t] = P.G[s][t];
  M.Gw = P.Gw;
  M.nu0 = P.nu0;
  M.nu_inf = P.nu_inf;
  M.lam = P.lam;
  M.K_d = P.K_d;
  M.rho_th = P.rho_th;
  M.w_theta = P.w_theta;
  M.xi_b = P.xi_b;
  M.xi_s = P.xi_s;
  M.rtol = P.newton_rtol;
  for (int s = 0; s < 2; ++s) {
    M.rho_in[s] = P.rho_in[s];
    M.rho_out[s] = P.rho_out[s];
  }
  return M;
}

template <typename T>
Ptrs<T> make_ptrs(elbm_ctx *c) {
  Ptrs<T> a;
  char *b = c->base;
  a.fa = (T *)(b + (c->parity ? c->o_fb : c->o_fa));
  a.fb = (T *)(b + (c->parity ? c->o_fa : c->o_fb));
  a.rho = (T *)(b + c->o_rho);
  a.psi = (T *)(b + c->o_psi);
  a.grad = (T *)(b + c->o_grad);
  a.bulk = (T *)(b + c->o_bulk);
  a.surf = (T *)(b + c->o_surf);
  a.q = (T *)(b + c->o_q);
  a.phi = (T *)(b + c->o_phi);
  a.rhs = (T *)(b + c->o_rhs);
  a.e2 = (T *)(b + c->o_e2);
  a.rec_u = (T *)(b + c->o_recu);
  a.rec_alpha = (double *)(b + c->o_reca);
  a.rec_iters = (int32_t *)(b + c->o_reci);
  a.type = (uint8_t *)(b + c->o_type);
  a.boxes = (const BoxDev *)(b + c->o_boxes);
  a.block_box = (const int32_t *)(b + c->o_bb);
  a.partials = (double *)(b + c->o_part);
  a.scal = (double *)(b + c->o_scal);
  a.cnt = (unsigned long long *)(b + c->o_cnt);
  a.err = (uint32_t *)(b + c->o_err);
  a.N = c->Ntot;
  return a;
}

double *stage(elbm_ctx *c, int plane) { return (double *)(c->base + c->o_stage) + (int64_t)plane * c->maxN; }

// Records the next timing event of the current step (no-op when timing is off).
elbm_status mark(elbm_ctx *c, hipEvent_t *evs, int k) {
  if (!c->timing) return ELBM_OK;
  HIPCHK(c, hipEventRecord(evs[k], c->stream));
  return ELBM_OK;
}

// Folds the recorded events of every timed step into phase_ms.
elbm_status collect_timing(elbm_ctx *c) {
  const size_t per = ELBM_NPHASES + 1;
  for (size_t s = 0; s + per <= c->ev_used; s += per) {
    for (int k = 0; k < ELBM_NPHASES; ++k) {
      float ms = 0.f;
      HIPCHK(c, hipEventElapsedTime(&ms, c->ev_pool[s + k], c->ev_pool[s + k + 1]));
      c->phase_ms[k] += ms;
    }
    c->timed_steps += 1;
  }
  c->ev_used = 0;
  return ELBM_OK;
}

template <typename T, int C>
elbm_status launch_steps(elbm_ctx *c, int nsteps, int record) {
  const Model M = make_model(c->P);
  const dim3 grid(c->nblocks), blk(BLK);
  const int nb = (int)c->boxes.size();
  for (int it = 0; it < nsteps; ++it) {
    Ptrs<T> a = make_ptrs<T>(c);
    const int rec = record && (it == nsteps - 1);
    hipEvent_t *ev = nullptr;
    if (c->timing) {
      const size_t per = ELBM_NPHASES + 1;
      if (c->ev_used + per > 6000) {  // bound the pool: fold what is recorded so far
        HIPCHK(c, hipStreamSynchronize(c->stream));
        elbm_status st = collect_timing(c);
        if (st) return st;
      }
      while (c->ev_pool.size() < c->ev_used + per) {
        hipEvent_t e;
        HIPCHK(c, hipEventCreate(&e));
        c->ev_pool.push_back(e);
      }
      ev = c->ev_pool.data() + c->ev_used;
      c->ev_used += per;
    }
    mark(c, ev, 0);
    hipLaunchKernelGGL((k_density<T, C>), grid, blk, 0, c->stream, a);
    mark(c, ev, 1);
    hipLaunchKernelGGL((k_gradient<T>), grid, blk, 0, c->stream, a);
    hipLaunchKernelGGL((k_interface<T>), grid, blk, 0, c->stream, a, M);
    hipLaunchKernelGGL(k_charge_coef, dim3(nb), blk, 0, c->stream, a.boxes, a.partials, a.scal, M);
    hipLaunchKernelGGL((k_charge_rhs<T>), grid, blk, 0, c->stream, a);
    mark(c, ev, 2);
    for (int sw = 0; sw < c->P.sor_sweeps; ++sw) {
      hipLaunchKernelGGL((k_sor<T>), grid, blk, 0, c->stream, a, 0);
      hipLaunchKernelGGL((k_sor<T>), grid, blk, 0, c->stream, a, 1);
    }
    if (c->any_gauge) {
      hipLaunchKernelGGL((k_phi_partials<T>), grid, blk, 0, c->stream, a);
      hipLaunchKernelGGL(k_phi_mean, dim3(nb), blk, 0, c->stream, a.boxes, a.partials, a.scal);
      hipLaunchKernelGGL((k_phi_sub<T>), grid, blk, 0, c->stream, a);
    }
    mark(c, ev, 3);
    hipLaunchKernelGGL((k_efield<T>), grid, blk, 0, c->stream, a);
    mark(c, ev, 4);
    hipLaunchKernelGGL((k_collide<T, C>), grid, blk, 0, c->stream, a, M, rec);
    mark(c, ev, 5);
    c->parity ^= 1;
  }
  HIPCHK(c, hipGetLastError());
  return ELBM_OK;
}

template <typename T>
elbm_status set_box_impl(elbm_ctx *c, int box, const uint8_t *type, const double *rho,
                         const double *u, const double *phi, const double *u_bc, const double *xi,
                         double jitter) {
  const BoxDev &B = c->bdev[box];
  const int C = c->P.ncomp;
  const size_t nb = (size_t)B.n;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(c->base + c->o_type + B.off, type, nb, hipMemcpyHostToDevice));
  // stage planes: rho [C], u [3], u_bc [3], xi (one at a time)
  for (int s = 0; s < C; ++s)
    HIPCHK(c, hipMemcpy(stage(c, s), rho + s * nb, nb * 8, hipMemcpyHostToDevice));
  for (int d = 0; d < 3; ++d) {
    if (u) HIPCHK(c, hipMemcpy(stage(c, 2 + d), u + d * nb, nb * 8, hipMemcpyHostToDevice));
    else HIPCHK(c, hipMemset(stage(c, 2 + d), 0, nb * 8));
    if (u_bc) HIPCHK(c, hipMemcpy(stage(c, 5 + d), u_bc + d * nb, nb * 8, hipMemcpyHostToDevice));
  }
  Ptrs<T> a = make_ptrs<T>(c);
  const Model M = make_model(c->P);
  const dim3 grid((unsigned)((B.n + BLK - 1) / BLK)), blk(BLK);
  for (int s = 0; s < C; ++s)
    for (int p = 0; p < NQ; ++p) {
      const double *xp = nullptr;
      if (xi) {
        HIPCHK(c, hipMemcpy(stage(c, 8), xi + ((size_t)s * NQ + p) * nb, nb * 8, hipMemcpyHostToDevice));
        xp = stage(c, 8);
      }
      hipLaunchKernelGGL((k_init_dir<T>), grid, blk, 0, c->stream, a, M, box, s, p, stage(c, 0), stage(c, 2),
                         u_bc ? stage(c, 5) : nullptr, xp, jitter, c->maxN);
      HIPCHK(c, hipGetLastError());
      HIPCHK(c, hipStreamSynchronize(c->stream));
    }
  // potential
  if (phi) {
    HIPCHK(c, hipMemcpy(stage(c, 0), phi, nb * 8, hipMemcpyHostToDevice));
    hipLaunchKernelGGL((k_from_double<T>), grid, blk, 0, c->stream, stage(c, 0),
                       (T *)(c->base + c->o_phi) + B.off, (T *)nullptr, B.n);
  } else {
    HIPCHK(c, hipMemset(c->base + c->o_phi + B.off * sizeof(T), 0, nb * sizeof(T)));
  }
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return ELBM_OK;
}

template <typename T>
elbm_status read_planes(elbm_ctx *c, int box, size_t field_off, int nplanes, double *host) {
  const BoxDev &B = c->bdev[box];
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const dim3 grid((unsigned)((B.n + BLK - 1) / BLK)), blk(BLK);
  for (int k = 0; k < nplanes; ++k) {
    const T *src = (const T *)(c->base + field_off) + (int64_t)k * c->Ntot + B.off;
    hipLaunchKernelGGL((k_to_double<T>), grid, blk, 0, c->stream, src, stage(c, 0), B.n);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(host + (size_t)k * B.n, stage(c, 0), (size_t)B.n * 8, hipMemcpyDeviceToHost));
  }
  return ELBM_OK;
}

template <typename T>
elbm_status write_planes(elbm_ctx *c, int box, size_t off1, size_t off2, int nplanes, const double *host) {
  const BoxDev &B = c->bdev[box];
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const dim3 grid((unsigned)((B.n + BLK - 1) / BLK)), blk(BLK);
  for (int k = 0; k < nplanes; ++k) {
    HIPCHK(c, hipMemcpy(stage(c, 0), host + (size_t)k * B.n, (size_t)B.n * 8, hipMemcpyHostToDevice));
    T *d1 = (T *)(c->base + off1) + (int64_t)k * c->Ntot + B.off;
    T *d2 = off2 ? (T *)(c->base + off2) + (int64_t)k * c->Ntot + B.off : nullptr;
    hipLaunchKernelGGL((k_from_double<T>), grid, blk, 0, c->stream, stage(c, 0), d1, d2, B.n);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return ELBM_OK;
}

elbm_status check_box_arg(elbm_ctx *c, int box) {
  if (!c) return ELBM_EINVAL;
  if (!c->bound) return fail(c, ELBM_ESTATE, "context is not bound to an arena");
  if (box < 0 || box >= (int)c->boxes.size()) return fail(c, ELBM_EINVAL, "box index out of range");
  return ELBM_OK;
}

size_t cur_pop_off(const elbm_ctx *c) { return c->parity ? c->o_fb : c->o_fa; }

}  // namespace

extern "C" {

uint32_t elbm_abi_version(void) { return ELBM_ABI_VERSION; }

elbm_status elbm_create(const elbm_params *P, const elbm_box *boxes, int32_t nboxes, elbm_ctx **out) {
  if (!out) return ELBM_EINVAL;
  *out = nullptr;
  if (!P || !boxes || nboxes <= 0) return ELBM_EINVAL;
  if (P->ncomp < 1 || P->ncomp > 2) return ELBM_EINVAL;
  if (P->storage != ELBM_STORAGE_F64 && P->storage != ELBM_STORAGE_F32) return ELBM_EINVAL;
  if (P->sor_sweeps < 0 || P->newton_max < 1 || P->newton_max > 1000) return ELBM_EINVAL;
  if (P->charge_model != ELBM_CHARGE_CONSERVING && P->charge_model != ELBM_CHARGE_GENERATOR) return ELBM_EINVAL;
  if (!(P->w_theta > 0.0) || !(P->K_d > 0.0) || !(P->nu0 > 0.0) || !(P->newton_rtol > 0.0)) return ELBM_EINVAL;
  if (P->carreau && !(P->nu_inf > 0.0 && P->lam >= 0.0)) return ELBM_EINVAL;
  if (P->alpha_guess != ELBM_GUESS_STANDARD) return ELBM_EINVAL;
  elbm_ctx *c = new (std::nothrow) elbm_ctx();
  if (!c) return ELBM_ENOMEM;
  c->P = *P;
  c->esz = P->storage == ELBM_STORAGE_F64 ? 8 : 4;
  int64_t off = 0;
  int blk0 = 0;
  for (int b = 0; b < nboxes; ++b) {
    const elbm_box &x = boxes[b];
    if (x.nx < 2 || x.ny < 2 || x.nz < 2) { delete c; return ELBM_EINVAL; }
    const int64_t n = (int64_t)x.nx * x.ny * x.nz;
    if (n > (int64_t)1 << 30) { delete c; return ELBM_EINVAL; }
    const int nn[3] = {x.nx, x.ny, x.nz};
    for (int d = 0; d < 3; ++d)
      if (x.periodic[d] && (nn[d] & 1)) { delete c; return ELBM_EINVAL; }  // red-black needs even periods
    if (!(x.sor_omega > 0.0 && x.sor_omega < 2.0)) { delete c; return ELBM_EINVAL; }
    if (P->carreau && !(x.n_flow > 0.0)) { delete c; return ELBM_EINVAL; }
    BoxDev d{};
    d.off = off;
    d.nx = x.nx; d.ny = x.ny; d.nz = x.nz; d.n = (int32_t)n;
    for (int k = 0; k < 3; ++k) { d.per[k] = x.periodic[k] ? 1 : 0; d.E[k] = x.E_ext[k]; }
    d.Q_b = x.Q_b; d.Q_s = x.Q_s; d.n_flow = x.n_flow; d.omega = x.sor_omega;
    const int nblk = (int)((n + BLK - 1) / BLK);
    d.first_block = blk0;
    d.nblocks = nblk;
    c->bdev.push_back(d);
    c->boxes.push_back(x);
    for (int i = 0; i < nblk; ++i) c->block_box.push_back(b);
    blk0 += nblk;
    off += (int64_t)nblk * BLK;
    if (n > c->maxN) c->maxN = n;
  }
  c->Ntot = off;
  c->nblocks = blk0;
  const int C = P->ncomp;
  const int64_t N = c->Ntot;
  const size_t e = c->esz;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
  c->o_fa = take((size_t)C * NQ * N * e);
  c->o_fb = take((size_t)C * NQ * N * e);
  c->o_rho = take((size_t)C * N * e);
  c->o_psi = take((size_t)C * N * e);
  c->o_grad = take(3 * (size_t)N * e);
  c->o_bulk = take((size_t)N * e);
  c->o_surf = take((size_t)N * e);
  c->o_q = take((size_t)N * e);
  c->o_phi = take((size_t)N * e);
  c->o_rhs = take((size_t)N * e);
  c->o_e2 = take((size_t)N * e);
  c->o_recu = take(3 * (size_t)N * e);
  c->o_reca = take((size_t)C * N * 8);
  c->o_reci = take((size_t)C * N * 4);
  c->o_type = take((size_t)N);
  c->o_stage = take(9 * (size_t)c->maxN * 8);
  c->o_boxes = take(sizeof(BoxDev) * nboxes);
  c->o_bb = take(sizeof(int32_t) * c->nblocks);
  c->o_part = take(sizeof(double) * 4 * (size_t)c->nblocks);
  c->o_scal = take(sizeof(double) * NSCAL * nboxes);
  c->o_cnt = take(sizeof(unsigned long long) * NCNT * nboxes);
  c->o_err = take(sizeof(uint32_t) * 4);
  c->total = o;
  *out = c;
  return ELBM_OK;
}

elbm_status elbm_required_bytes(const elbm_ctx *c, size_t *bytes) {
  if (!c || !bytes) return ELBM_EINVAL;
  *bytes = c->total;
  return ELBM_OK;
}

elbm_status elbm_bind(elbm_ctx *c, void *arena, size_t bytes, void *stream) {
  if (!c) return ELBM_EINVAL;
  if (!arena || ((uintptr_t)arena & 255)) return fail(c, ELBM_EINVAL, "arena must be non-null and 256-byte aligned");
  if (bytes < c->total) return fail(c, ELBM_ENOMEM, "arena smaller than elbm_required_bytes");
  c->base = (char *)arena;
  c->stream = (hipStream_t)stream;
  c->parity = 0;
  c->any_gauge = false;
  // Dirichlet flags come with the node types; assume none until set_box
  for (auto &d : c->bdev) { d.has_dirichlet = 0; d.n_unknown = d.n; }
  for (auto &d : c->bdev) if (!d.has_dirichlet) c->any_gauge = true;
  HIPCHK(c, hipMemcpy(c->base + c->o_boxes, c->bdev.data(), sizeof(BoxDev) * c->bdev.size(), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->base + c->o_bb, c->block_box.data(), sizeof(int32_t) * c->block_box.size(), hipMemcpyHostToDevice));
  // zero every field once: padding nodes stay solid (type 1) and inert
  HIPCHK(c, hipMemset(c->base, 0, c->o_type));
  HIPCHK(c, hipMemset(c->base + c->o_type, K_SOLID, (size_t)c->Ntot));
  HIPCHK(c, hipMemset(c->base + c->o_scal, 0, c->total - c->o_scal));
  c->bound = true;
  return ELBM_OK;
}

elbm_status elbm_set_box(elbm_ctx *c, int32_t box, const uint8_t *type, const double *rho, const double *u,
                         const double *phi, const double *u_bc, const double *xi, double jitter) {
  elbm_status st = check_box_arg(c, box);
  if (st) return st;
  if (!type || !rho) return fail(c, ELBM_EINVAL, "node_type and rho are required");
  BoxDev &B = c->bdev[box];
  int64_t nu = 0;
  bool dir = false;
  for (int i = 0; i < B.n; ++i) {
    if (type[i] > 7) return fail(c, ELBM_EINVAL, "node type byte out of range");
    if (type[i] & B_DIRICHLET) dir = true; else ++nu;
  }
  B.has_dirichlet = dir ? 1 : 0;
  B.n_unknown = (int32_t)nu;
  c->any_gauge = false;
  for (auto &d : c->bdev) if (!d.has_dirichlet) c->any_gauge = true;
  HIPCHK(c, hipMemcpy(c->base + c->o_boxes + sizeof(BoxDev) * box, &B, sizeof(BoxDev), hipMemcpyHostToDevice));
  if (c->P.storage == ELBM_STORAGE_F64) return set_box_impl<double>(c, box, type, rho, u, phi, u_bc, xi, jitter);
  return set_box_impl<float>(c, box, type, rho, u, phi, u_bc, xi, jitter);
}

elbm_status elbm_step(elbm_ctx *c, int32_t nsteps, int32_t record) {
  if (!c) return ELBM_EINVAL;
  if (!c->bound) return fail(c, ELBM_ESTATE, "context is not bound to an arena");
  if (nsteps < 0) return fail(c, ELBM_EINVAL, "nsteps must be >= 0");
  if (nsteps == 0) return ELBM_OK;
  const bool f64 = c->P.storage == ELBM_STORAGE_F64;
  if (c->P.ncomp == 2) return f64 ? launch_steps<double, 2>(c, nsteps, record) : launch_steps<float, 2>(c, nsteps, record);
  return f64 ? launch_steps<double, 1>(c, nsteps, record) : launch_steps<float, 1>(c, nsteps, record);
}

elbm_status elbm_sync(elbm_ctx *c) {
  if (!c) return ELBM_EINVAL;
  if (!c->bound) return fail(c, ELBM_ESTATE, "context is not bound to an arena");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  uint32_t e = 0;
  HIPCHK(c, hipMemcpy(&e, c->base + c->o_err, sizeof(e), hipMemcpyDeviceToHost));
  if (e & 1u) return fail(c, ELBM_ENONFINITE, "a post-collision population became non-finite");
  return ELBM_OK;
}

elbm_status elbm_read_moments(elbm_ctx *c, int32_t box, double *rho, double *u) {
  elbm_status st = check_box_arg(c, box);
  if (st) return st;
  const bool f64 = c->P.storage == ELBM_STORAGE_F64;
  if (rho) {
    st = f64 ? read_planes<double>(c, box, c->o_rho, c->P.ncomp, rho) : read_planes<float>(c, box, c->o_rho, c->P.ncomp, rho);
    if (st) return st;
  }
  if (u) st = f64 ? read_planes<double>(c, box, c->o_recu, 3, u) : read_planes<float>(c, box, c->o_recu, 3, u);
  return st;
}

elbm_status elbm_read_potential(elbm_ctx *c, int32_t box, double *phi) {
  elbm_status st = check_box_arg(c, box);
  if (st) return st;
  if (!phi) return fail(c, ELBM_EINVAL, "phi is NULL");
  return c->P.storage == ELBM_STORAGE_F64 ? read_planes<double>(c, box, c->o_phi, 1, phi)
                                          : read_planes<float>(c, box, c->o_phi, 1, phi);
}

elbm_status elbm_read_charge(elbm_ctx *c, int32_t box, double *q) {
  elbm_status st = check_box_arg(c, box);
  if (st) return st;
  if (!q) return fail(c, ELBM_EINVAL, "q is NULL");
  return c->P.storage == ELBM_STORAGE_F64 ? read_planes<double>(c, box, c->o_q, 1, q)
                                          : read_planes<float>(c, box, c->o_q, 1, q);
}

elbm_status elbm_read_alpha(elbm_ctx *c, int32_t box, double *alpha, int32_t *iters) {
  elbm_status st = check_box_arg(c, box);
  if (st) return st;
  const BoxDev &B = c->bdev[box];
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int s = 0; s < c->P.ncomp; ++s) {
    if (alpha)
      HIPCHK(c, hipMemcpy(alpha + (size_t)s * B.n, (double *)(c->base + c->o_reca) + (int64_t)s * c->Ntot + B.off,
                          (size_t)B.n * 8, hipMemcpyDeviceToHost));
    if (iters)
      HIPCHK(c, hipMemcpy(iters + (size_t)s * B.n, (int32_t *)(c->base + c->o_reci) + (int64_t)s * c->Ntot + B.off,
                          (size_t)B.n * 4, hipMemcpyDeviceToHost));
  }
  return ELBM_OK;
}

elbm_status elbm_get_populations(elbm_ctx *c, int32_t box, double *f) {
  elbm_status st = check_box_arg(c, box);
  if (st) return st;
  if (!f) return fail(c, ELBM_EINVAL, "f is NULL");
  const int np = c->P.ncomp * NQ;
  return c->P.storage == ELBM_STORAGE_F64 ? read_planes<double>(c, box, cur_pop_off(c), np, f)
                                          : read_planes<float>(c, box, cur_pop_off(c), np, f);
}

elbm_status elbm_set_populations(elbm_ctx *c, int32_t box, const double *f) {
  elbm_status st = check_box_arg(c, box);
  if (st) return st;
  if (!f) return fail(c, ELBM_EINVAL, "f is NULL");
  const int np = c->P.ncomp * NQ;
  const size_t other = c->parity ? c->o_fa : c->o_fb;
  return c->P.storage == ELBM_STORAGE_F64 ? write_planes<double>(c, box, cur_pop_off(c), other, np, f)
                                          : write_planes<float>(c, box, cur_pop_off(c), other, np, f);
}

elbm_status elbm_set_potential(elbm_ctx *c, int32_t box, const double *phi) {
  elbm_status st = check_box_arg(c, box);
  if (st) return st;
  if (!phi) return fail(c, ELBM_EINVAL, "phi is NULL");
  return c->P.storage == ELBM_STORAGE_F64 ? write_planes<double>(c, box, c->o_phi, 0, 1, phi)
                                          : write_planes<float>(c, box, c->o_phi, 0, 1, phi);
}

elbm_status elbm_diagnostics(elbm_ctx *c, int32_t box, elbm_diag *out) {
  elbm_status st = check_box_arg(c, box);
  if (st) return st;
  if (!out) return fail(c, ELBM_EINVAL, "out is NULL");
  memset(out, 0, sizeof(*out));
  const BoxDev &B = c->bdev[box];
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const int nblk = (B.n + BLK - 1) / BLK;
  const dim3 grid(nblk), blk(BLK);
  double *dst = stage(c, 0);
  const bool f64 = c->P.storage == ELBM_STORAGE_F64;
  if (f64) {
    Ptrs<double> a = make_ptrs<double>(c);
    if (c->P.ncomp == 2) hipLaunchKernelGGL((k_diag<double, 2>), grid, blk, 0, c->stream, a, box, dst);
    else hipLaunchKernelGGL((k_diag<double, 1>), grid, blk, 0, c->stream, a, box, dst);
  } else {
    Ptrs<float> a = make_ptrs<float>(c);
    if (c->P.ncomp == 2) hipLaunchKernelGGL((k_diag<float, 2>), grid, blk, 0, c->stream, a, box, dst);
    else hipLaunchKernelGGL((k_diag<float, 1>), grid, blk, 0, c->stream, a, box, dst);
  }
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::vector<double> part((size_t)nblk * 5);
  HIPCHK(c, hipMemcpy(part.data(), dst, part.size() * 8, hipMemcpyDeviceToHost));
  for (int i = 0; i < nblk; ++i) {
    out->mass[0] += part[i * 5 + 0];
    out->mass[1] += part[i * 5 + 1];
    for (int d = 0; d < 3; ++d) out->momentum[d] += part[i * 5 + 2 + d];
  }
  unsigned long long cn[NCNT];
  HIPCHK(c, hipMemcpy(cn, c->base + c->o_cnt + sizeof(unsigned long long) * NCNT * box, sizeof(cn), hipMemcpyDeviceToHost));
  out->n_fallback = (int64_t)cn[0];
  out->n_negative = (int64_t)cn[2];
  out->n_collisions = (int64_t)cn[4];
  const int64_t solved = (int64_t)cn[4] - (int64_t)cn[0];
  out->mean_newton_iters = solved > 0 ? (double)cn[1] / (double)solved : 0.0;
  // alpha statistics of the last recorded step over fluid nodes
  std::vector<double> al((size_t)B.n);
  std::vector<uint8_t> ty((size_t)B.n);
  HIPCHK(c, hipMemcpy(ty.data(), c->base + c->o_type + B.off, (size_t)B.n, hipMemcpyDeviceToHost));
  double mn = INFINITY, mx = -INFINITY, sm = 0.0;
  int64_t cntn = 0;
  for (int s = 0; s < c->P.ncomp; ++s) {
    HIPCHK(c, hipMemcpy(al.data(), (double *)(c->base + c->o_reca) + (int64_t)s * c->Ntot + B.off, (size_t)B.n * 8,
                        hipMemcpyDeviceToHost));
    for (int i = 0; i < B.n; ++i)
      if ((ty[i] & 3) == K_FLUID) {
        mn = fmin(mn, al[i]);
        mx = fmax(mx, al[i]);
        sm += al[i];
        ++cntn;
      }
  }
  out->alpha_min = cntn ? mn : 0.0;
  out->alpha_max = cntn ? mx : 0.0;
  out->alpha_mean = cntn ? sm / (double)cntn : 0.0;
  return ELBM_OK;
}

elbm_status elbm_set_timing(elbm_ctx *c, int32_t enable) {
  if (!c) return ELBM_EINVAL;
  if (!c->bound) return fail(c, ELBM_ESTATE, "context is not bound to an arena");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->timing = enable != 0;
  c->ev_used = 0;
  for (double &v : c->phase_ms) v = 0.0;
  c->timed_steps = 0;
  return ELBM_OK;
}

elbm_status elbm_timing(elbm_ctx *c, double *ms, int64_t *steps) {
  if (!c) return ELBM_EINVAL;
  if (!c->bound) return fail(c, ELBM_ESTATE, "context is not bound to an arena");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  elbm_status st = collect_timing(c);
  if (st) return st;
  if (ms)
    for (int k = 0; k < ELBM_NPHASES; ++k) ms[k] = c->phase_ms[k];
  if (steps) *steps = c->timed_steps;
  for (double &v : c->phase_ms) v = 0.0;
  c->timed_steps = 0;
  return ELBM_OK;
}

const char *elbm_last_error(const elbm_ctx *c) {
  if (!c) return "null context";
  return c->err.c_str();
}

void elbm_destroy(elbm_ctx *c) { delete c; }

}  // extern "C"
