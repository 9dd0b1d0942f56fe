// elbm_device.h -- device-side tables, data structures and per-node maths of
// the entropic lattice Boltzmann update for charged leaky-dielectric
// multiphase fluids (Lauricella et al., arXiv:1612.05404), for gfx950.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "elbm.h"

namespace elbm {

constexpr int NQ = 19;
constexpr int BLK = 256;
constexpr int K_FLUID = 0, K_SOLID = 1, K_INLET = 2, K_OUTLET = 3, B_DIRICHLET = 4, B_NOZZLE = 8;

// D3Q19 velocity set (order documented in elbm.h).
constexpr int kCx[NQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int kCy[NQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int kCz[NQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

// weights: the paper's D2Q9 set 4/9, 1/9, 1/36 lifted to D3Q19 (same c_s^2 = 1/3)
__host__ __device__ constexpr double wgt(int p) {
  return p == 0 ? 1.0 / 3.0 : (p < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
}
__host__ __device__ constexpr int opp(int p) { return p == 0 ? 0 : ((p & 1) ? p + 1 : p - 1); }

// Lattice descriptors, the template parameter L of every kernel that walks
// the velocity set.  D3Q19 (the 3-D lift, order in elbm.h) and D2Q9, the
// paper's own lattice (Sec. II): rest, +x, -x, +y, -y, (+1,+1), (-1,-1),
// (+1,-1), (-1,+1), weights 4/9, 1/9, 1/36, c_s^2 = 1/3; a D2Q9 box is one
// x-y plane (nz = 1, bounded in z).  Opposite directions sit at adjacent
// (odd, even) indices in both, so opp() serves both.
struct D3Q19 {
  static constexpr int Q = 19, D = 3;
  static constexpr int cx[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  static constexpr int cy[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  static constexpr int cz[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  __host__ __device__ static constexpr double w(int p) { return wgt(p); }
};
struct D2Q9 {
  static constexpr int Q = 9, D = 2;
  static constexpr int cx[Q] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
  static constexpr int cy[Q] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
  static constexpr int cz[Q] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  __host__ __device__ static constexpr double w(int p) {
    return p == 0 ? 4.0 / 9.0 : (p < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
  }
};
constexpr int QMAX = 19;

constexpr double CS2 = 1.0 / 3.0;

struct BoxDev {
  int64_t off;          // first arena node of the box
  int32_t nx, ny, nz, n;
  int32_t per[3];
  int32_t has_dirichlet;
  int32_t first_block, nblocks, n_unknown, pad;
  double E[3];
  double Q_b, Q_s, n_flow, omega;
  double rnx, rny;  // 1/nx, 1/ny (FP64) for the index division of div_extent
};

struct Model {
  int32_t C, carreau, curvature, electrostriction, charge_model, newton_max, alpha_guess, strict;
  int32_t alpha_iter, sor_check_every;
  int32_t inlet_mode;  // ELBM_INLET_*
  double G[2][2], Gw[2][2], nu0, nu_inf, lam, K_d, rho_th, w_theta, xi_b, xi_s, rtol;
  double rho_in[2], rho_out[2];
  double sor_tol;
};

// scalars per box: [0] charge scale of the bulk part, [1] of the surface
// part, [2] neutralising charge qbar, [3] mean potential, [4] Poisson
// residual of the last check, [5] its scale max|rhs|, [6] sweeps done at
// that check, [7] 1 once this step's solve has met its tolerance, [8] mean
// velocity inside the nozzle (adaptive inlet)
constexpr int NSCAL = 9;
// counters per box: fallbacks, Newton updates, negative f, non-finite f,
// collisions, Poisson solves above their tolerance
constexpr int NCNT = 8;
// bits of the sticky error word
constexpr uint32_t ERR_NONFINITE = 1u, ERR_NEGPOP = 2u, ERR_ALPHA = 4u, ERR_SOR = 8u;

// T: population storage type, F: field storage / stencil arithmetic type
template <typename T, typename F>
struct Ptrs {
  T *fa, *fb;           // populations: read fa, write fb
  F *rho, *psi, *grad, *bulk, *surf, *q, *phi, *rhs, *e2;  // psi [N][C]; grad: unit normal [3], |grad rho_A|^2
  F *rec_u;
  const F *ubc;         // [3][N] inlet velocity (read at inlet nodes)
  double *ab;           // [C][N] alpha * beta of the step's collision
  double *rec_alpha;
  int32_t *rec_iters;
  uint8_t *type;
  const uint32_t *nbm;   // [N] bit p: neighbour r + c_p solid or outside the box (static geometry)
  const BoxDev *boxes;
  const int32_t *block_box;
  double *partials;     // [nblocks][4]
  double *res_part;     // [nblocks][2] Poisson residual and max|rhs| per block
  double *fel_part;     // [nblocks][3] electric force summed per block (recorded steps)
  double *noz_part;     // [nblocks][2] momentum along the inlet axis and mass of NOZZLE nodes per block
  double *scal;         // [nboxes][NSCAL]
  unsigned long long *cnt;  // [nboxes][NCNT]
  uint32_t *err;
  int64_t N;            // arena nodes (plane stride)
  int32_t nblocks;      // node blocks of one launch
  int32_t remap;        // 1: XCD-aware block order
  int32_t prio;         // 1: field-chain waves beside k_alpha at raised issue priority
  // block tiles of the collision (tx = 0: 256 consecutive nodes per block)
  const int32_t *tile_box;  // [ntiles] box of each tile
  const int4 *box_tiles;    // [nboxes] first tile, tiles along x, y, z
  int32_t tx, ty, tz, ntiles;
};

// Block tile shapes of the collision, index 1..: the 256 threads cover
// tx x ty x tz nodes, x fastest, so each 64-thread wave is a 3-D patch
// (8x8x1, 8x4x2, 4x4x4); index 0 is the linear mapping.
constexpr int NTILE_SHAPES = 4;
__host__ __device__ constexpr int tile_dim(int shape, int axis) {
  return shape == 1 ? (axis == 0 ? 8 : axis == 1 ? 8 : 4)
       : shape == 2 ? (axis == 0 ? 8 : axis == 1 ? 4 : 8)
       : shape == 3 ? (axis == 0 ? 4 : axis == 1 ? 4 : 16) : 0;
}

// The field-chain kernels after the densities (gradient, interface, charge,
// SOR sweeps, gauge, E field) run beside k_alpha, which keeps two long
// FP64-bound waves on every SIMD. With prio set their waves get a higher
// instruction-issue priority, so that these short, latency-bound kernels
// issue first (worth it where the chain is the longer branch); it changes no
// result. Called after a kernel's uniform loads: the compiler treats the
// priority instruction as a side effect and turns the scalar (uniform) loads
// that follow it into vector loads.
__device__ __forceinline__ void field_chain_priority(int prio) {
  if (prio) __builtin_amdgcn_s_setprio(3);
}

// ------------------------------------------------------------ node decode
struct Node {
  BoxDev B;
  int bb, blk;  // box, logical block
  int64_t g;
  int n, x, y, z;
  bool live;
};

// Logical block of this workgroup.  Workgroups go to the 8 XCDs round-robin;
// with remap, XCD k runs one contiguous range of logical blocks, so tiles
// that share halos share an L2.  A bijection of [0, nb).
__device__ __forceinline__ int logical_block(int nb, int remap) {
  const int b = blockIdx.x;
  if (!remap) return b;
  const int q = nb >> 3, r = nb & 7, k = b & 7, i = b >> 3;
  return (k < r ? k * (q + 1) : r * (q + 1) + (k - r) * q) + i;
}

// Node of this thread in the tiled mapping (a.tx > 0).  Threads of a tile
// beyond the box edge are not live (their coordinates are the tile corner's).
template <typename P>
__device__ __forceinline__ void decode_tile(const P &a, Node &nd) {
  nd.blk = logical_block(a.ntiles, a.remap);
  nd.bb = a.tile_box[nd.blk];
  nd.B = a.boxes[nd.bb];
  const int4 bt = a.box_tiles[nd.bb];
  const int lt = nd.blk - bt.x;
  const int bx = lt % bt.y, r = lt / bt.y, by = r % bt.z, bz = r / bt.z;
  const int t = threadIdx.x, r2 = t / a.tx;
  const int x = bx * a.tx + t % a.tx, y = by * a.ty + r2 % a.ty, z = bz * a.tz + r2 / a.ty;
  nd.live = x < nd.B.nx && y < nd.B.ny && z < nd.B.nz;
  nd.x = nd.live ? x : bx * a.tx;
  nd.y = nd.live ? y : by * a.ty;
  nd.z = nd.live ? z : bz * a.tz;
  nd.n = nd.x + nd.B.nx * (nd.y + nd.B.ny * nd.z);
  nd.g = nd.B.off + nd.n;
}

// t / n for 0 <= t < 2^30 and an extent n >= 1 from rn = 1/n (FP64), in
// place of an integer division: (t + 1/2)/n lies at least 1/(2n) from an
// integer, and the two roundings (of 1/n and of the product) move it by at
// most (t + 1/2)/n * 2^-52 < 2^-22/n, so the truncation is the exact quotient.
__host__ __device__ __forceinline__ int div_extent(int t, double rn) { return (int)((double(t) + 0.5) * rn); }

template <typename P>
__device__ __forceinline__ void decode(const P &a, Node &nd) {
  nd.blk = logical_block(a.nblocks, a.remap);
  nd.bb = a.block_box[nd.blk];
  nd.B = a.boxes[nd.bb];
  nd.g = (int64_t)nd.blk * BLK + threadIdx.x;
  nd.n = (int)(nd.g - nd.B.off);
  nd.live = nd.n < nd.B.n;
  const int t = nd.live ? nd.n : 0;
  const int r = div_extent(t, nd.B.rnx);
  nd.x = t - r * nd.B.nx;
  nd.z = div_extent(r, nd.B.rny);
  nd.y = r - nd.z * nd.B.ny;
}

// One axis of nbr: the coordinate c + d wrapped once by the extent n where
// the axis is periodic; ok cleared where it leaves a closed axis.
__host__ __device__ __forceinline__ int wrap_axis(int c, int d, int n, int per, bool &ok) {
  const int v = c + d;
  if (d == 0) return v;  // a lattice offset: resolved at compile time in the unrolled loops
  const bool lo = v < 0, hi = v >= n;
  ok &= !(lo | hi) | (per != 0);
  return lo ? v + n : hi ? v - n : v;
}

// local index of r + (dx,dy,dz), wrapping periodic axes; -1 outside the box.
// Selects only, no branches: in the unrolled stencil loops a branch per
// direction and axis cost more than the loads it guarded.
__host__ __device__ __forceinline__ int nbr(const BoxDev &B, int x, int y, int z, int dx, int dy, int dz) {
  bool ok = true;
  const int xx = wrap_axis(x, dx, B.nx, B.per[0], ok);
  const int yy = wrap_axis(y, dy, B.ny, B.per[1], ok);
  const int zz = wrap_axis(z, dz, B.nz, B.per[2], ok);
  const int m = xx + B.nx * (yy + B.ny * zz);
  return ok ? m : -1;
}

// --------------------------------------------------------- reductions
// Fixed-order block sum of K doubles (64-lane wave butterflies, then the
// four waves in order): bitwise reproducible run to run.
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

// Block maxima of K non-negative doubles (waves, then the four wave results).
template <int K>
__device__ __forceinline__ void block_max_store(double (&v)[K], double *out) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = fmax(v[k], __shfl_xor(v[k], off, 64));
  __shared__ double sm[BLK / 64][K];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) sm[wid][k] = v[k];
  __syncthreads();
  if (threadIdx.x < K) {
    double s = sm[0][threadIdx.x];
#pragma unroll
    for (int w = 1; w < BLK / 64; ++w) s = fmax(s, sm[w][threadIdx.x]);
    out[threadIdx.x] = s;
  }
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// -------------------------------------------------------- equilibrium
// Second-order equilibrium (Sec. II, below Eq. lattice-b), with the exact
// lattice factors 1/c_s^2 = 3 and 1/(2 c_s^4) = 4.5 (no divisions):
// w rho [1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u.u].
// c.u with the lattice vector's components (0 or +-1) folded in: zero
// components add no term (an FMA with a zero coefficient is not folded away
// under IEEE rules), unit ones add or subtract.
template <typename R>
__device__ __forceinline__ R cdot(int cx, int cy, int cz, R ux, R uy, R uz) {
  R cu = R(0);
  bool first = true;
  if (cx) { cu = cx > 0 ? ux : -ux; first = false; }
  if (cy) { cu = first ? (cy > 0 ? uy : -uy) : (cy > 0 ? cu + uy : cu - uy); first = false; }
  if (cz) { cu = first ? (cz > 0 ? uz : -uz) : (cz > 0 ? cu + uz : cu - uz); }
  return cu;
}
template <typename Lat, typename R>
__device__ __forceinline__ R feq(int p, R rho, R ux, R uy, R uz, R uu) {
  const R cu = cdot<R>(Lat::cx[p], Lat::cy[p], Lat::cz[p], ux, uy, uz);
  return R(Lat::w(p)) * rho * (R(1) + R(3) * cu + R(4.5) * (cu * cu) - R(1.5) * uu);
}

// 1/d to ~1 ulp: hardware reciprocal estimate refined by two Newton steps.
__device__ __forceinline__ double rcp_nr(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(fma(-d, r, 1.0), r, r);
  return fma(fma(-d, r, 1.0), r, r);
}

// ln(1 + y) for y > -1 to ~2 ulp (the libm version carries double-double
// internals and is ~5x longer).  t = 1 + y with its exact rounding error c
// (TwoSum); t = m 2^e with m in [1/sqrt2, sqrt2); ln m = 2 atanh(s),
// s = (m-1)/(m+1), |s| <= 0.1716, summed as 2 s sum_{k=0}^{10} s^2k/(2k+1)
// (first dropped term 2e-17 relative); ln(1+y) = e ln2 + ln m + c/t.
__device__ __forceinline__ double log1p_fast(double y) {
  const double t = 1.0 + y;
  const double bv = t - 1.0, av = t - bv;
  const double c = (1.0 - av) + (y - bv);
  double m = __builtin_amdgcn_frexp_mant(t);
  int e = __builtin_amdgcn_frexp_exp(t);
  if (m < 0.70710678118654752440) {
    m *= 2.0;
    e -= 1;
  }
  const double s = (m - 1.0) * rcp_nr(m + 1.0);
  const double s2 = s * s;
  double q = 1.0 / 21.0;
  q = fma(q, s2, 1.0 / 19.0);
  q = fma(q, s2, 1.0 / 17.0);
  q = fma(q, s2, 1.0 / 15.0);
  q = fma(q, s2, 1.0 / 13.0);
  q = fma(q, s2, 1.0 / 11.0);
  q = fma(q, s2, 1.0 / 9.0);
  q = fma(q, s2, 1.0 / 7.0);
  q = fma(q, s2, 1.0 / 5.0);
  q = fma(q, s2, 1.0 / 3.0);
  q = fma(q, s2, 1.0);
  const double de = double(e);
  // ln2 split: the high part has 33 significant bits, so de * LN2_HI is exact
  return fma(de, 6.93147180369123816490e-01, fma(de, 1.90821492927058770002e-10, 2.0 * s * q + c * __builtin_amdgcn_rcp(t)));
}

// e^x for |x| < 700 to ~2 ulp: x = k ln2 + r with the same split of ln2 as
// log1p_fast (k ln2_hi exact), |r| <= ln2/2, e^r by its Taylor series through
// r^13 (first dropped term below 3e-18 relative), then the power of two.
__device__ __forceinline__ double exp_fast(double x) {
  const double k = rint(x * 1.44269504088896340736);
  const double r = fma(-k, 1.90821492927058770002e-10, fma(-k, 6.93147180369123816490e-01, x));
  double p = 1.0 / 6227020800.0;
  p = fma(p, r, 1.0 / 479001600.0);
  p = fma(p, r, 1.0 / 39916800.0);
  p = fma(p, r, 1.0 / 3628800.0);
  p = fma(p, r, 1.0 / 362880.0);
  p = fma(p, r, 1.0 / 40320.0);
  p = fma(p, r, 1.0 / 5040.0);
  p = fma(p, r, 1.0 / 720.0);
  p = fma(p, r, 1.0 / 120.0);
  p = fma(p, r, 1.0 / 24.0);
  p = fma(p, r, 1.0 / 6.0);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p, int(k));
}

// (1 + q)^e for q >= 0, the Carreau factor: e^(e ln(1 + q)) in FP64 (no
// rounding of 1 + q), the library pow in FP32.  For q < 2^-10 (a shear rate
// well below 1/lambda: most of a flow at rest) both factors are short
// Taylor series: ln(1 + q) through q^6 and e^t, |t| = |e| q < 2e-3, through
// t^6 (dropped terms below 2e-19 relative).
template <typename R>
__device__ __forceinline__ R pow1p(R q, R e) {
  if constexpr (sizeof(R) == 8) {
    if (q < 0.0009765625) {
      double l = -1.0 / 6.0;
      l = fma(l, q, 1.0 / 5.0);
      l = fma(l, q, -1.0 / 4.0);
      l = fma(l, q, 1.0 / 3.0);
      l = fma(l, q, -0.5);
      l = fma(l, q, 1.0);
      const double t = e * (l * q);
      double x = 1.0 / 720.0;
      x = fma(x, t, 1.0 / 120.0);
      x = fma(x, t, 1.0 / 24.0);
      x = fma(x, t, 1.0 / 6.0);
      x = fma(x, t, 0.5);
      x = fma(x, t, 1.0);
      return fma(x, t, 1.0);
    }
    return exp_fast(e * log1p_fast(q));
  } else {
    return pow(R(1) + q, e);
  }
}

// phi(y) = (1+y) ln(1+y) - y given l = ln(1+y), cancellation-free: Taylor
// series sum_{k>=2} (-1)^k y^k / (k(k-1)) through k = 15 for |y| < 1/16
// (first dropped term below 2e-19 relative), the closed form elsewhere.
__device__ __forceinline__ double phi_of(double y, double l) {
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
  return (1.0 + y) * l - y;
}

// Entropic alpha (Eqs. entropic, H): the non-trivial root of
//   g(a) = sum_p f_p phi(a x_p) + a L,  x = (f_eq - f)/f,  L = sum_p Delta_p ln(f_p / (w_p rho)),
// which equals H(f + a Delta) - H(f) exactly (sum Delta = 0).  L is formed
// as sum_p Delta_p log1p((f_p - w_p rho)/(w_p rho)) (one log per direction,
// no cancellation).  g is convex on the positivity interval (0, a_max) with
// g(0) = 0, g'(0) = L, and finite at a_max (the vanishing population adds
// f_p phi(-1) = f_p): a root exists iff L < 0 and g(a_max-) > 0.
// Starters: 2 (ELBM_GUESS_STANDARD); the series starter (ELBM_GUESS_SERIES),
// the root of the degree-11 truncation (SERIES_DEG) of
// g(a)/a = L + sum_k (-1)^k a^(k-1) M_k / (k(k-1)), M_k = sum_p f_p x_p^k,
// accepted inside the positivity interval while a0 max|x| < SERIES_ACCEPT
// (beyond 0.2 the truncation is no longer small, but up to about 1 the root
// is still a closer start than 2: fewer updates at interface nodes); the
// learned starter (ELBM_GUESS_MLP) takes the series starter where it is
// accepted and the network's a0 where it is not (and a0 lies in the
// positivity interval).  Every starter is polished by Newton to the same
// stopping rule.  At an accepted series root b the rule can hold without an
// evaluation of g: with q the truncated series, g(b)/b - q(b) is the series
// tail from degree 12, bounded by b^11 M_12 / (132 (1 - b max|x|)) for
// b max|x| < 1, and S(b) >= b^2 M_2 (1 - b max|x|/3) / 2 (phi(y) >= y^2/2 -
// |y|^3/6).  When b (|q(b)| + tail) <= rtol S_lower / 2, the evaluation would
// accept b with 0 updates, so b is returned directly.  Likewise after a plain
// Newton step d from a: by Taylor, |g(a + d)| <= g''_max d^2 / 2 with
// g'' = sum f x^2 / (1 + xi x) <= M_2 / D, D = 1 - max(a, a + d) / a_max, and
// S(a + d) >= S(a) - |d| max(a, a + d) M_2 / D; within half the tolerance the
// evaluation at a + d would accept it, so it is returned without one.  The update count goes to `iters`, or -1 with the fallback
// min(2, 0.99 a_max) when there is no root, Newton does not converge, or a
// population is not positive (H undefined).
// The set-up runs in two passes over the directions: x_p, max|x| and the
// positivity bound, then the moments with L.  Between them the wave picks the
// series degree: when every node of the wave has max|x| < QUIET_X (fluid near
// equilibrium, most of a flow) the degree-5 truncation already meets the
// acceptance bound and needs six moments instead of twelve, and its
// logarithms take the Taylor path for small arguments (log1p_near0).
// f: the node's 19 populations of one component (thread-private LDS column,
// element p at offset p * BLK); xs: scratch for x (element p at p * XSTRIDE
// in the wave's own LDS block).  Both keep the Newton loop rolled and the
// register footprint small.  rho, u: FP64 moments of f.
constexpr int XSTRIDE = 64;  // stride of a thread's x column in its wave's LDS block
constexpr double SERIES_ACCEPT = 1.2;

// State between the set-up pass and the Newton polish.
struct AlphaSetup {
  double L, amax, xmax, a;  // a: the starter so far
  double M2;                // sum_p f_p x_p^2
  int state;                // 0: Newton needed, 1: at equilibrium (2), 2: fallback, 3: the rule holds at a
  bool want_learned;        // the learned starter would be used here
};

// Degree of the series starter's truncation: moments M_2 .. M_{D+1} (the last
// one for the tail bound).  Measured on the e-field drop: 7 lets 23 % of the
// liquid component's waves skip Newton, 11 lets 67 % (alpha kernel 5 % faster),
// 15 lets 83 % but costs more in the set-up pass than it saves.
constexpr int SERIES_DEG = 11;

// The truncated series q(b) = L + sum_{k=2}^{D} (-1)^k b^(k-1) M_k / (k(k-1))
// (g(b)/b without its tail) and its derivative in b, by Horner's rule
// (M[k - 2] = M_k).
template <int D>
__device__ __forceinline__ double series_q(double b, double L, const double *M) {
  double h = ((D & 1) ? -M[D - 2] : M[D - 2]) / double(D * (D - 1));
#pragma unroll
  for (int k = D - 1; k >= 2; --k) h = fma(b, h, ((k & 1) ? -M[k - 2] : M[k - 2]) / double(k * (k - 1)));
  return fma(b, h, L);
}
template <int D>
__device__ __forceinline__ double series_dq(double b, const double *M) {
  double h = ((D & 1) ? -M[D - 2] : M[D - 2]) / double(D);
#pragma unroll
  for (int k = D - 1; k >= 2; --k) h = fma(b, h, ((k & 1) ? -M[k - 2] : M[k - 2]) / double(k));
  return h;
}

// ln(1 + y) for |y| < 1/32 by its Taylor series through y^12 (first dropped
// term below 3e-19 relative, no reciprocal), log1p_fast elsewhere.
__device__ __forceinline__ double log1p_near0(double y) {
  if (fabs(y) < 0.03125) {
    double h = -1.0 / 12.0;
    h = fma(h, y, 1.0 / 11.0);
    h = fma(h, y, -1.0 / 10.0);
    h = fma(h, y, 1.0 / 9.0);
    h = fma(h, y, -1.0 / 8.0);
    h = fma(h, y, 1.0 / 7.0);
    h = fma(h, y, -1.0 / 6.0);
    h = fma(h, y, 1.0 / 5.0);
    h = fma(h, y, -1.0 / 4.0);
    h = fma(h, y, 1.0 / 3.0);
    h = fma(h, y, -0.5);
    return fma(h * y, y, y);
  }
  return log1p_fast(y);
}

// Degree of the series starter on quiet waves (every node with max|x| below
// QUIET_X): there the degree-5 truncation already meets the acceptance bound
// at b ~ 2 (tail b^5 M_6 / 30 <= 2^3 max|x|^4 b^2 M_2 / 30), so its six
// moments replace the twelve of SERIES_DEG.
constexpr int QUIET_DEG = 5;
constexpr double QUIET_X = 5e-4;

// Moments M_2 .. M_{D+1} of one node from its x and f columns and the
// entropy term L = sum_p Delta_p ln(f_p / (w_p rho)) (fixed order p = 0..Q-1;
// Delta_p = x_p f_p, from the stored x_p = Delta_p / f_p rather than a second
// evaluation of the equilibrium: the same to rounding).  NEAR0: the logarithm
// takes its Taylor series where |y| < 1/32.
template <typename Lat, typename T, int D, bool NEAR0>
__device__ __forceinline__ double series_moments(const T *f, const double *xs, double *M, double rho, double irho) {
#pragma unroll
  for (int k = 0; k < D; ++k) M[k] = 0.0;
  double L = 0.0;
#pragma unroll
  for (int p = 0; p < Lat::Q; ++p) {
    const double fp = double(f[p * BLK]);
    const double x = xs[p * XSTRIDE];
    double t = fp * x * x;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      M[k] += t;
      t *= x;
    }
    const double wr = Lat::w(p) * rho;
    const double d = x * fp;
    const double y = (fp - wr) * (irho * (1.0 / Lat::w(p)));
    L += d * (NEAR0 ? log1p_near0(y) : log1p_fast(y));
  }
  return L;
}

// Newton on the degree-D truncated series from 2 (no logarithms); sets
// st.a / st.state / st.want_learned as the series starter decides.
template <int D>
__device__ __forceinline__ void series_start(AlphaSetup &st, const double *M, double L, double amax,
                                             double xmax, int guess, double rtol) {
  double b = 2.0;
#pragma unroll 1
  for (int k = 0; k < 6; ++k) {
    const double q = series_q<D>(b, L, M);
    const double dq = series_dq<D>(b, M);
    if (!(dq > 0.0)) break;
    const double step = q / dq;
    b -= step;
    if (fabs(step) <= 1e-15 * b) break;  // converged: further updates move b by rounding only
  }
  if (b > 0.0 && b < amax && b * xmax < SERIES_ACCEPT) {
    st.a = b;
    const double bx = b * xmax;
    if (bx < 0.5) {
      const double qb = series_q<D>(b, L, M);
      double bd = b;  // b^D
#pragma unroll
      for (int k = 1; k < D; ++k) bd *= b;
      const double tail = bd * M[D - 1] / (double((D + 1) * D) * (1.0 - bx));
      if (b * (fabs(qb) + tail) <= 0.25 * rtol * b * b * M[0] * (1.0 - bx / 3.0)) st.state = 3;
    }
  } else {
    st.want_learned = guess == ELBM_GUESS_MLP;
  }
}


template <typename Lat, typename T>
__device__ __forceinline__ AlphaSetup alpha_setup(const T *f, double *xs, double rho, double ux, double uy,
                                                  double uz, int guess, double rtol) {
  const double uu = ux * ux + uy * uy + uz * uz;
  const double irho = rcp_nr(rho);
  double xmax = 0.0, xmin = 0.0;
  bool nonpos = false;
#pragma unroll  // fully: the lattice vectors fold into the equilibria
  for (int p = 0; p < Lat::Q; ++p) {
    const double fp = double(f[p * BLK]);
    const double d = feq<Lat, double>(p, rho, ux, uy, uz, uu) - fp;
    const double x = d * rcp_nr(fp);
    nonpos |= !(fp > 0.0);
    xs[p * XSTRIDE] = x;
    xmax = fmax(xmax, fabs(x));
    xmin = fmin(xmin, x);
  }
  // top of the positivity interval, min over x_p < 0 of -1/x_p = -1/min x
  const double amax = xmin < 0.0 ? -rcp_nr(xmin) : INFINITY;
  AlphaSetup st;
  st.L = 0.0;
  st.amax = amax;
  st.xmax = xmax;
  st.a = 2.0;
  st.want_learned = false;
  st.M2 = 0.0;
  if (nonpos) {  // H(f) is undefined for a non-positive population
    st.state = 2;
    return st;
  }
  const bool series = guess == ELBM_GUESS_SERIES || guess == ELBM_GUESS_MLP;
  // the moments the series starter and the Taylor bounds need, at the
  // degree of the wave: quiet waves (every active lane near equilibrium)
  // take the short truncation
  double M[SERIES_DEG];
  const bool quiet = series && __all(xmax < QUIET_X);
  double L;
  if (quiet) L = series_moments<Lat, T, QUIET_DEG, true>(f, xs, M, rho, irho);
  else if (series) L = series_moments<Lat, T, SERIES_DEG, false>(f, xs, M, rho, irho);
  else L = series_moments<Lat, T, 1, false>(f, xs, M, rho, irho);
  st.L = L;
  st.M2 = M[0];
  if (xmax < 1e-12) {
    st.state = 1;
    return st;
  }
  st.state = L < 0.0 ? 0 : 2;
  if (st.state == 0 && series) {
    if (quiet) series_start<QUIET_DEG>(st, M, L, amax, xmax, guess, rtol);
    else series_start<SERIES_DEG>(st, M, L, amax, xmax, guess, rtol);
  }
  return st;
}

// Newton's starting point for a node that needs the iteration (state 0).
__device__ __forceinline__ double alpha_start(const AlphaSetup &st, double a0) {
  double a = st.a;
  if (st.want_learned && a0 > 0.0 && a0 < st.amax) a = a0;
  if (!(a > 0.0 && a < st.amax)) a = 0.5 * fmin(st.amax, 4.0);
  return a;
}

// g at the top of the positivity interval, g(amax-) = sum_p f_p phi(amax x_p)
// + amax L, where the population that vanishes contributes f_p phi(-1) = f_p:
// with L < 0 a root exists in (0, amax) iff this is positive.
template <typename Lat, typename T>
__device__ __forceinline__ double alpha_g_top(const T *f, const double *xs, double L, double amax) {
  double S = 0.0;
#pragma unroll 1
  for (int p = 0; p < Lat::Q; ++p) {
    const double y = amax * xs[p * XSTRIDE];
    S += double(f[p * BLK]) * (y > -1.0 ? phi_of(y, log1p_fast(y)) : 1.0);
  }
  return S + amax * L;
}

// Newton (or Halley) on g from a inside (0, amax) (f, xs as for the set-up
// pass).  The first step that would leave the interval at the top checks that
// a root exists at all (alpha_g_top); none: the fallback at once.  Halley's
// step a - (g / g') / (1 - h), h = g g'' / (2 g'^2), uses
// g'' = sum_p f_p x_p^2 / (1 + a x_p) (one reciprocal per direction, no
// logarithm); it is taken while |h| < 1/2 (at most twice the Newton step),
// else the Newton step: next to a_max a nearly vanishing population makes
// g'' large, h approaches 1 and the unguarded step leaves the interval and
// cycles.  The Taylor bound that skips the final evaluation holds for
// Newton steps only.
template <typename Lat, typename T>
__device__ __forceinline__ double alpha_iterate(const T *f, const double *xs, double L, double amax, double M2,
                                                double a, double rtol, int maxit, int &iters, bool halley) {
  {
    bool probed = false;
    for (int it = 0; it <= maxit; ++it) {
      double S = 0.0, gp = L, gpp = 0.0;
#pragma unroll 4
      for (int p = 0; p < Lat::Q; ++p) {
        const double fp = double(f[p * BLK]);
        const double x = xs[p * XSTRIDE];
        const double y = a * x;
        const double l = log1p_fast(y);
        S += fp * phi_of(y, l);
        gp += (x * fp) * l;
        if (halley) gpp += (x * fp) * x * rcp_nr(1.0 + y);
      }
      const double g = S + a * L;
      if (fabs(g) <= rtol * S) {
        iters = it;
        return a;
      }
      if (it == maxit) break;
      double an = (gp > 0.0) ? a - g / gp : 2.0 * a;
      bool newton = gp > 0.0 && an > 0.0 && an < amax;
      if (halley && gp > 0.0) {
        const double h = g * gpp / (2.0 * gp * gp);
        if (fabs(h) < 0.5) {
          an = a - (g / gp) / (1.0 - h);
          newton = false;
        }
      }
      if (an >= amax) {
        if (!probed) {
          probed = true;
          if (!(alpha_g_top<Lat, T>(f, xs, L, amax) > 0.0)) break;
        }
        an = 0.5 * (a + amax);
        newton = false;
      }
      if (an <= 0.0) {
        an = 0.5 * a;
        newton = false;
      }
      if (fabs(an - a) <= 4.0 * 2.220446049250313e-16 * a) {
        iters = it + 1;
        return an;
      }
      if (newton) {  // Taylor bound at the Newton point (see above)
        const double d = an - a, hi = fmax(a, an), D = 1.0 - hi / amax;
        if (D > 0.0) {
          const double G2 = M2 / D;
          if (G2 * d * d <= rtol * (S - fabs(d) * hi * G2)) {
            iters = it + 1;
            return an;
          }
        }
      }
      a = an;
    }
  }
  iters = -1;
  return fmin(2.0, 0.99 * amax);
}

template <typename Lat, typename T>
__device__ __forceinline__ double alpha_newton(const T *f, const double *xs, AlphaSetup st, double a0, double rtol,
                                               int maxit, int &iters, bool halley = false) {
  if (st.state == 1 || st.state == 3) {
    iters = 0;
    return st.state == 1 ? 2.0 : st.a;
  }
  if (st.state == 0)
    return alpha_iterate<Lat, T>(f, xs, st.L, st.amax, st.M2, alpha_start(st, a0), rtol, maxit, iters, halley);
  iters = -1;
  return fmin(2.0, 0.99 * st.amax);
}

// Input of the learned starter from the x_p of the set-up pass: with
// r_p = f_p / f_eq_p = 1/(1 + x_p), z_p = (r_p - 1)/s (z[0..18]) and
// s = max_p |r_p - 1|.  Valid when every f_eq_p is positive (x_p > -1) and
// 0 < s <= 1.
__device__ __forceinline__ bool features_from_x(const double *xs, float *z, double &scale) {
  double r[NQ];
  bool ok = true;
  double sc = 0.0;
#pragma unroll
  for (int p = 0; p < NQ; ++p) {
    const double x = xs[p * XSTRIDE];
    ok &= x > -1.0;
    r[p] = -x * rcp_nr(1.0 + x);
    sc = fmax(sc, fabs(r[p]));
  }
  ok &= (sc > 0.0) && (sc <= 1.0);
  const double is = ok ? rcp_nr(sc) : 0.0;
#pragma unroll
  for (int p = 0; p < NQ; ++p) z[p] = ok ? float(r[p] * is) : 0.0f;
  scale = sc;
  return ok;
}

// Matrix 2-norm of a symmetric 3x3 (largest |eigenvalue|), cyclic Jacobi
// rotations until the off-diagonal part is below 1e-12 of the diagonal
// (squared: 1e-24; the eigenvalues then carry an error of second order in
// it, far below rounding).  In FP64 the rotation (Rutishauser's form) uses
// the refined hardware reciprocal and reciprocal square root instead of
// divisions and square roots: a rotation accurate to ~1 ulp is orthogonal to
// rounding, which is all the eigenvalues need.
__device__ __forceinline__ double rsq_nr(double d) {
  double r = __builtin_amdgcn_rsq(d);
  const double h = 0.5 * d;
  r = r * fma(-h * r, r, 1.5);
  return r * fma(-h * r, r, 1.5);
}

template <typename R>
__device__ R sym3_norm2_jacobi(R a00, R a11, R a22, R a01, R a02, R a12) {
  R a[3][3] = {{a00, a01, a02}, {a01, a11, a12}, {a02, a12, a22}};
  const R tiny = sizeof(R) == 8 ? R(1e-24) : R(1e-14);
  for (int sweep = 0; sweep < 10; ++sweep) {
    const R off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    const R diag = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
    if (off <= tiny * diag || off == R(0)) break;
#pragma unroll
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
      if (a[p][q] == R(0)) continue;
      R t, c;
      if constexpr (sizeof(R) == 8) {
        const double th = (a[q][q] - a[p][p]) * rcp_nr(2.0 * a[p][q]);
        const double at = fabs(th);
        // |th| beyond 1e100: t = 1/(2 th) to full precision, and th^2 would overflow
        const double tm = at > 1e100 ? 0.5 * rcp_nr(at) : rcp_nr(at + (th * th + 1.0) * rsq_nr(th * th + 1.0));
        t = th >= 0.0 ? tm : -tm;
        c = rsq_nr(t * t + 1.0);
      } else {
        const R th = (a[q][q] - a[p][p]) / (R(2) * a[p][q]);
        t = (th >= R(0) ? R(1) : R(-1)) / (fabs(th) + sqrt(th * th + R(1)));
        c = R(1) / sqrt(t * t + R(1));
      }
      const R s = t * c;
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

// The same 2-norm from the characteristic cubic: with q = tr A / 3,
// B = (A - q I) / p, p^2 = tr((A - q I)^2) / 6, the eigenvalues are
// q + 2 p cos(phi + 2 pi k / 3), phi = acos(det B / 2) / 3 in [0, pi/3].  c =
// cos(phi) is the largest root of 4 c^3 - 3 c = r, r = det B / 2: an FP32
// start from acos / cos, then two Newton steps in R; sin(phi) =
// sqrt(1 - c^2).  The largest eigenvalue is q + 2 p c, the smallest
// q - p (c + sqrt3 sin(phi)), the middle one 3q minus those.  Near a double
// eigenvalue (|r| -> 1) the cubic's roots lose digits (error ~ eps /
// sqrt(1 - r^2)), so for 1 - |r| < 5e-5 the Jacobi iteration above answers.
// Elsewhere the result is within ~1e-14 relative of the exact 2-norm.
template <typename R>
__device__ R sym3_norm2(R a00, R a11, R a22, R a01, R a02, R a12) {
  const R p1 = a01 * a01 + a02 * a02 + a12 * a12;
  const R q = (a00 + a11 + a22) * R(1.0 / 3.0);
  const R b00 = a00 - q, b11 = a11 - q, b22 = a22 - q;
  const R p2 = b00 * b00 + b11 * b11 + b22 * b22 + R(2) * p1;
  if (!(p2 > R(0))) return fabs(q);
  R p, ip;
  if constexpr (sizeof(R) == 8) {
    const double h = p2 * (1.0 / 6.0);
    const double rs = rsq_nr(h);
    p = h * rs;
    ip = rs;
  } else {
    p = sqrt(p2 * R(1.0 / 6.0));
    ip = R(1) / p;
  }
  const R c00 = b00 * ip, c11 = b11 * ip, c22 = b22 * ip, c01 = a01 * ip, c02 = a02 * ip, c12 = a12 * ip;
  const R r = R(0.5) * (c00 * (c11 * c22 - c12 * c12) - c01 * (c01 * c22 - c12 * c02) + c02 * (c01 * c12 - c11 * c02));
  if (!(fabs(r) < R(1) - R(5e-5))) return sym3_norm2_jacobi<R>(a00, a11, a22, a01, a02, a12);
  R c = R(cosf(acosf(float(r)) * (1.0f / 3.0f)));
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const R g = (R(4) * c * c - R(3)) * c - r;
    const R dg = R(12) * c * c - R(3);
    if constexpr (sizeof(R) == 8) c -= g * rcp_nr(dg);
    else c -= g / dg;
  }
  const R s2 = R(1) - c * c;
  R sn;
  if constexpr (sizeof(R) == 8) sn = s2 > 0.0 ? s2 * rsq_nr(s2) : 0.0;
  else sn = sqrt(fmax(s2, R(0)));
  const R l1 = q + R(2) * p * c;
  const R l3 = q - p * (c + R(1.7320508075688772935) * sn);
  const R l2 = R(3) * q - l1 - l3;
  return fmax(fabs(l1), fmax(fabs(l2), fabs(l3)));
}

// Shear rate of Eq. strain2: the root of h(g) = rho (2 nu(g) + c_s^2) g - alpha Pi
// (Carreau nu, Eq. carreau).  nu0 >= nu >= nu_inf brackets it between the
// Newtonian roots of the two limits; Newton from the nu0 end, kept inside the
// bracket (h is strictly increasing for n > 0).
// Pi = 0 or rho <= 0 (reachable only after negative populations): no
// positive root, the shear rate is 0 (nu = nu0).
template <typename R>
__device__ R shear_rate(R Pn, R rho, R alpha, R nu0, R ninf, R lam, R n) {
  if (!(Pn > R(0)) || !(rho > R(0))) return R(0);
  R lo = alpha * Pn / (rho * (R(2) * nu0 + R(CS2)));
  R hi = alpha * Pn / (rho * (R(2) * ninf + R(CS2)));
  R g = lo;
  const R tol = sizeof(R) == 8 ? R(1e-15) : R(2e-7);
  for (int it = 0; it < 60; ++it) {
    const R lg = lam * g;
    const R s = R(1) + lg * lg;
    const R e = pow1p<R>(lg * lg, R(0.5) * (n - R(3)));  // s^((n-3)/2); s^((n-1)/2) = s * e
    const R nu = ninf + (nu0 - ninf) * s * e;
    const R h = rho * (R(2) * nu + R(CS2)) * g - alpha * Pn;
    if (h > R(0)) hi = g; else lo = g;
    const R dh = rho * (R(2) * ninf + R(CS2) + R(2) * (nu0 - ninf) * e * (R(1) + n * lg * lg));
    R gn = g - h / dh;
    const bool newton = gn >= lo && gn <= hi;
    if (!newton) gn = R(0.5) * (lo + hi);
    if (fabs(gn - g) <= tol * g || hi - lo <= tol * R(0.1) * hi) return gn;
    // a Newton step this small is in the quadratic regime: the next update
    // would be below the tolerance (relative 1e-16), so gn is returned now
    if (sizeof(R) == 8 && newton && fabs(gn - g) <= R(1e-8) * g) return gn;
    g = gn;
  }
  return g;
}

}  // namespace elbm
