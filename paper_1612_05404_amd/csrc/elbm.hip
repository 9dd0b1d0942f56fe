// elbm.hip -- C ABI (include/elbm.h) of the gfx950 library for the
// per-time-step update of the entropic lattice Boltzmann model for charged
// leaky-dielectric multiphase fluids (Lauricella et al., arXiv:1612.05404).
//
// Data layout in HBM (one arena owned by the caller):
//   all boxes of a context are concatenated node-wise; every box starts at a
//   multiple of 256 nodes (padding nodes are typed solid and never updated),
//   so a 256-thread block always lies inside one box.  Every field is
//   structure-of-arrays with one plane of Ntot nodes per component /
//   direction / vector axis: f[(s*19 + p)*Ntot + g], x fastest inside a box.
//   Populations are double buffered (pull from one, write the other, swap).
//   Storage: populations in T, auxiliary fields (densities, psi, gradient,
//   charge weights, charge, potential, |E|^2) in F:
//     ELBM_STORAGE_F64      T = F = double
//     ELBM_STORAGE_F32      T = float, F = double
//     ELBM_STORAGE_F32_ALL  T = F = float
//   The entropic alpha and the collision moments are FP64 in every mode.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "elbm.h"
#include "elbm_kernels.h"

using namespace elbm;

// ====================================================================== ABI
struct elbm_ctx {
  elbm_params P;
  std::vector<elbm_box> boxes;
  std::vector<BoxDev> bdev;
  std::vector<int32_t> block_box;
  int64_t Ntot = 0;
  int64_t maxN = 0;
  int Q = 19;  // directions of the context's lattice
  int nblocks = 0;
  size_t esz_pop = 8, esz_fld = 8;
  // arena offsets (bytes)
  size_t o_fa, o_fb, o_rho, o_psi, o_grad, o_bulk, o_surf, o_q, o_phi, o_rhs, o_e2, o_recu, o_ubc, o_ab, o_nbm, o_reca,
      o_reci, o_type, o_stage, o_boxes, o_bb, o_part, o_rpart, o_fpart, o_npart, o_scal, o_cnt, o_err, total;
  // learned alpha starter: FP32 master + Adam moments, BF16 matrices, gradient, partials, losses
  size_t o_mp, o_mm, o_mv, o_mw1, o_mw2, o_mw2t, o_mgrad, o_mpart, o_mloss;
  int64_t adam_t = 0;
  int device = 0;  // the device current at bind (the arena's and the stream's)
  char *base = nullptr;
  hipStream_t stream = nullptr;
  // second stream for the alpha solve beside the field chain, and its fork/join events
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool bound = false;
  bool any_gauge = false;
  // SOR half sweeps with one thread per node pair: every box has an even x
  // extent and at least 2^20 nodes (measured faster there, slower on small
  // boxes where the pair's halved parallelism matters more)
  bool sor_pairs = false;
  // LDS slabs for the gradient and E-field stencils (launch option
  // stencil_lds): slab stride (0: they do not fit) and the dynamic LDS of one
  // block
  int slab_lmax = 0;
  size_t slab_bytes = 0;
  bool slabs = false;
  int parity = 0;  // which population buffer is current (0: fa region)
  std::string err;
  // device timing: ELBM_NPHASES + 1 events per timed step, recycled
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  double phase_ms[ELBM_NPHASES] = {0, 0, 0, 0, 0, 0};
  int64_t timed_steps = 0;
  // launch mapping: XCD-aware block order, steps per captured graph (even),
  // block tile shape of the collision (0: linear)
  int remap = 0;
  int graph_steps = 2;
  int prio = 0;  // issue priority of the field-chain waves beside k_alpha (0/1)
  int tile = 0;
  // per tile shape: tile -> box table, per-box tile counts, tiles in all
  std::vector<int32_t> tile_box[NTILE_SHAPES];
  std::vector<int4> box_tiles[NTILE_SHAPES];
  int ntiles[NTILE_SHAPES] = {0, 0, 0, 0};
  size_t o_tbox[NTILE_SHAPES] = {0, 0, 0, 0}, o_btiles[NTILE_SHAPES] = {0, 0, 0, 0};
  // captured step graphs, indexed by the starting population parity
  bool use_graphs = true;
  hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
  void drop_graphs() {
    for (hipGraphExec_t &g : graph_exec)
      if (g) {
        (void)hipGraphExecDestroy(g);
        g = nullptr;
      }
  }
  ~elbm_ctx() {
    drop_graphs();
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (aux) (void)hipStreamDestroy(aux);
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
  M.alpha_guess = P.alpha_guess;
  M.strict = P.strict;
  M.alpha_iter = P.alpha_iter;
  M.sor_check_every = P.sor_check_every;
  M.inlet_mode = P.inlet_mode;
  M.sor_tol = P.sor_tol;
  for (int s = 0; s < 2; ++s)
    for (int t = 0; t < 2; ++t) {
      M.G[s][t] = P.G[s][t];
      M.Gw[s][t] = P.Gw[s][t];
    }
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

template <typename T, typename F>
Ptrs<T, F> make_ptrs(elbm_ctx *c) {
  Ptrs<T, F> a;
  char *b = c->base;
  a.fa = (T *)(b + (c->parity ? c->o_fb : c->o_fa));
  a.fb = (T *)(b + (c->parity ? c->o_fa : c->o_fb));
  a.rho = (F *)(b + c->o_rho);
  a.psi = (F *)(b + c->o_psi);
  a.grad = (F *)(b + c->o_grad);
  a.bulk = (F *)(b + c->o_bulk);
  a.surf = (F *)(b + c->o_surf);
  a.q = (F *)(b + c->o_q);
  a.phi = (F *)(b + c->o_phi);
  a.rhs = (F *)(b + c->o_rhs);
  a.e2 = (F *)(b + c->o_e2);
  a.rec_u = (F *)(b + c->o_recu);
  a.ubc = (const F *)(b + c->o_ubc);
  a.ab = (double *)(b + c->o_ab);
  a.nbm = (const uint32_t *)(b + c->o_nbm);
  a.rec_alpha = (double *)(b + c->o_reca);
  a.rec_iters = (int32_t *)(b + c->o_reci);
  a.type = (uint8_t *)(b + c->o_type);
  a.boxes = (const BoxDev *)(b + c->o_boxes);
  a.block_box = (const int32_t *)(b + c->o_bb);
  a.partials = (double *)(b + c->o_part);
  a.res_part = (double *)(b + c->o_rpart);
  a.fel_part = (double *)(b + c->o_fpart);
  a.noz_part = (double *)(b + c->o_npart);
  a.scal = (double *)(b + c->o_scal);
  a.cnt = (unsigned long long *)(b + c->o_cnt);
  a.err = (uint32_t *)(b + c->o_err);
  a.N = c->Ntot;
  a.nblocks = c->nblocks;
  a.remap = c->remap;
  a.prio = c->prio;
  a.tile_box = (const int32_t *)(b + c->o_tbox[c->tile]);
  a.box_tiles = (const int4 *)(b + c->o_btiles[c->tile]);
  a.tx = tile_dim(c->tile, 0);
  a.ty = tile_dim(c->tile, 1);
  a.tz = tile_dim(c->tile, 2);
  a.ntiles = c->ntiles[c->tile];
  return a;
}

constexpr int MLP_MAX_STEPS = 4096;  // optimiser steps per elbm_mlp_train call

MlpDev make_mlp(elbm_ctx *c) {
  MlpDev W;
  W.w1 = (const __bf16 *)(c->base + c->o_mw1);
  W.w2 = (const __bf16 *)(c->base + c->o_mw2);
  W.w2t = (const __bf16 *)(c->base + c->o_mw2t);
  W.p = (const float *)(c->base + c->o_mp);
  return W;
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

// Enqueues one time step (every kernel of Sec. II.C) on the bound stream and
// flips the population parity.
template <typename Lat, typename T, typename F, int C>
elbm_status enqueue_step(elbm_ctx *c, int rec) {
  const Model M = make_model(c->P);
  const dim3 grid(c->nblocks), blk(BLK);
  const int nb = (int)c->boxes.size();
  Ptrs<T, F> a = make_ptrs<T, F>(c);
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
  // k_alpha needs only the populations: without phase timing it runs on the
  // second stream beside the rest of the field chain (gradient, interface,
  // charge, Poisson sweeps, E field), forked after the densities (beside the
  // density kernel too, the two pulls compete for HBM), and k_collide waits
  // for it; with timing everything runs in order on the bound stream.
  const dim3 cgrid(c->tile ? (unsigned)c->ntiles[c->tile] : grid.x);
  const bool fork = !c->timing;
  hipStream_t as = fork ? c->aux : c->stream;
  mark(c, ev, 0);
  hipLaunchKernelGGL((k_density<Lat, T, F, C>), grid, blk, 0, c->stream, a, c->P.inlet_mode - 1);
  mark(c, ev, 1);
  // the alpha kernel (the learned starter reads the 19 D3Q19 ratios)
  auto alpha_pass = [&]() {
    bool learned = false;
    if constexpr (Lat::Q == 19) {
      if (M.alpha_guess == ELBM_GUESS_MLP) {
        hipLaunchKernelGGL((k_alpha<Lat, T, F, C, true>), cgrid, blk, 0, as, a, M, make_mlp(c), rec);
        learned = true;
      }
    }
    if (!learned) hipLaunchKernelGGL((k_alpha<Lat, T, F, C, false>), cgrid, blk, 0, as, a, M, make_mlp(c), rec);
  };
  if (fork) {
    HIPCHK(c, hipEventRecord(c->ev_fork, c->stream));
    HIPCHK(c, hipStreamWaitEvent(c->aux, c->ev_fork, 0));
    alpha_pass();
    HIPCHK(c, hipEventRecord(c->ev_join, c->aux));
  }
  if (c->slabs)
    hipLaunchKernelGGL((k_gradient<Lat, T, F, true>), grid, blk, c->slab_bytes, c->stream, a, c->slab_lmax);
  else
    hipLaunchKernelGGL((k_gradient<Lat, T, F, false>), grid, blk, 0, c->stream, a, 0);
  hipLaunchKernelGGL((k_interface<Lat, T, F>), grid, blk, 0, c->stream, a, M);
  hipLaunchKernelGGL(k_charge_coef, dim3(nb), blk, 0, c->stream, a.boxes, a.partials, (const double *)a.noz_part,
                     a.scal, M, a.prio);
  hipLaunchKernelGGL((k_charge_rhs<T, F>), grid, blk, 0, c->stream, a);
  mark(c, ev, 2);
  // red-black sweeps; with a tolerance the FP64 residual is checked after
  // every sor_check_every sweeps (boxes within it skip the rest) and after
  // the last one, which recorded steps always take (diagnostics)
  const int nsw = c->P.sor_sweeps, every = c->P.sor_check_every;
  const bool tol = c->P.sor_tol > 0.0, checks = tol && every > 0;
  const dim3 pgrid((c->nblocks + 1) / 2);
  for (int sw = 1; sw <= nsw; ++sw) {
    if (c->sor_pairs) {
      hipLaunchKernelGGL((k_sor_pair<T, F>), pgrid, blk, 0, c->stream, a, 0, (int)checks);
      hipLaunchKernelGGL((k_sor_pair<T, F>), pgrid, blk, 0, c->stream, a, 1, (int)checks);
    } else {
      hipLaunchKernelGGL((k_sor<T, F>), grid, blk, 0, c->stream, a, 0, (int)checks);
      hipLaunchKernelGGL((k_sor<T, F>), grid, blk, 0, c->stream, a, 1, (int)checks);
    }
    if (checks && sw % every == 0 && sw < nsw) {
      hipLaunchKernelGGL((k_residual<T, F>), grid, blk, 0, c->stream, a, 1);
      hipLaunchKernelGGL(k_res_box, dim3(nb), blk, 0, c->stream, a.boxes, (const double *)a.res_part, a.scal, a.cnt,
                         a.err, c->P.sor_tol, sw, 0, a.prio);
    }
  }
  if (tol || rec) {
    hipLaunchKernelGGL((k_residual<T, F>), grid, blk, 0, c->stream, a, (int)checks);
    hipLaunchKernelGGL(k_res_box, dim3(nb), blk, 0, c->stream, a.boxes, (const double *)a.res_part, a.scal, a.cnt,
                       a.err, c->P.sor_tol, nsw, 1, a.prio);
  }
  if (c->any_gauge) {
    hipLaunchKernelGGL((k_phi_partials<T, F>), grid, blk, 0, c->stream, a);
    hipLaunchKernelGGL(k_phi_mean, dim3(nb), blk, 0, c->stream, a.boxes, a.partials, a.scal, a.prio);
    hipLaunchKernelGGL((k_phi_sub<T, F>), grid, blk, 0, c->stream, a);
  }
  mark(c, ev, 3);
  if (c->slabs)
    hipLaunchKernelGGL((k_efield<Lat, T, F, true>), grid, blk, c->slab_bytes, c->stream, a, c->slab_lmax);
  else
    hipLaunchKernelGGL((k_efield<Lat, T, F, false>), grid, blk, 0, c->stream, a, 0);
  mark(c, ev, 4);
  if (fork) {
    HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_join, 0));
  } else {
    alpha_pass();
  }
  mark(c, ev, 5);
  hipLaunchKernelGGL((k_collide<Lat, T, F, C>), grid, blk, 0, c->stream, a, M, rec);
  mark(c, ev, 6);
  c->parity ^= 1;
  HIPCHK(c, hipGetLastError());
  return ELBM_OK;
}

// nsteps steps.  Without per-phase timing, on a non-null stream, pairs of
// unrecorded steps replay a captured two-step hipGraph (one per starting
// parity, built on first use and kept with the context): the 2 x (7 + 2k)
// launches of a pair become one graph launch.
template <typename Lat, typename T, typename F, int C>
elbm_status launch_steps(elbm_ctx *c, int nsteps, int record) {
  int direct = nsteps;
  if (!c->timing && c->use_graphs && c->stream != nullptr) {
    const int k = c->graph_steps;  // even: a replay starts and ends at the same parity
    const int pairs = (record ? nsteps - 1 : nsteps) / k;
    if (pairs > 0) {
      hipGraphExec_t &ge = c->graph_exec[c->parity];
      if (!ge) {
        hipGraph_t g = nullptr;
        HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
        elbm_status s2 = ELBM_OK;
        for (int i = 0; i < k && !s2; ++i) s2 = enqueue_step<Lat, T, F, C>(c, 0);
        hipError_t ec = hipStreamEndCapture(c->stream, &g);
        if (s2) {
          if (g) (void)hipGraphDestroy(g);
          return s2;
        }
        if (ec != hipSuccess) return fail(c, ELBM_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
        hipError_t ei = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
          ge = nullptr;
          return fail(c, ELBM_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
        }
      }
      for (int i = 0; i < pairs; ++i) HIPCHK(c, hipGraphLaunch(ge, c->stream));
      direct = nsteps - k * pairs;
    }
  }
  for (int it = 0; it < direct; ++it) {
    elbm_status st = enqueue_step<Lat, T, F, C>(c, record && it == direct - 1);
    if (st) return st;
  }
  return ELBM_OK;
}

template <typename Lat, typename T, typename F>
elbm_status set_box_impl(elbm_ctx *c, int box, const uint8_t *type, const double *rho,
                         const double *u, const double *phi, const double *u_bc, const double *xi,
                         double jitter) {
  const BoxDev &B = c->bdev[box];
  const int C = c->P.ncomp;
  const size_t nb = (size_t)B.n;
  HIPCHK(c, hipMemcpy(c->base + c->o_type + B.off, type, nb, hipMemcpyHostToDevice));
  // stage planes: rho [C], u [3], u_bc [3], xi (one at a time)
  for (int s = 0; s < C; ++s)
    HIPCHK(c, hipMemcpy(stage(c, s), rho + s * nb, nb * 8, hipMemcpyHostToDevice));
  for (int d = 0; d < 3; ++d) {
    if (u) HIPCHK(c, hipMemcpy(stage(c, 2 + d), u + d * nb, nb * 8, hipMemcpyHostToDevice));
    else HIPCHK(c, hipMemset(stage(c, 2 + d), 0, nb * 8));
    if (u_bc) HIPCHK(c, hipMemcpy(stage(c, 5 + d), u_bc + d * nb, nb * 8, hipMemcpyHostToDevice));
  }
  Ptrs<T, F> a = make_ptrs<T, F>(c);
  const Model M = make_model(c->P);
  const dim3 grid((unsigned)((B.n + BLK - 1) / BLK)), blk(BLK);
  for (int s = 0; s < C; ++s)
    for (int p = 0; p < Lat::Q; ++p) {
      const double *xp = nullptr;
      if (xi) {
        HIPCHK(c, hipMemcpy(stage(c, 8), xi + ((size_t)s * Lat::Q + p) * nb, nb * 8, hipMemcpyHostToDevice));
        xp = stage(c, 8);
      }
      hipLaunchKernelGGL((k_init_dir<Lat, T, F>), grid, blk, 0, c->stream, a, M, box, s, p, stage(c, 0), stage(c, 2),
                         u_bc ? stage(c, 5) : nullptr, xp, jitter, c->maxN);
      HIPCHK(c, hipGetLastError());
      HIPCHK(c, hipStreamSynchronize(c->stream));
    }
  // neighbour masks (static geometry), for every box: cheap, and boxes set later redo them
  hipLaunchKernelGGL((k_neighbour_mask<Lat, T, F>), dim3(c->nblocks), blk, 0, c->stream, a,
                     (uint32_t *)(c->base + c->o_nbm));
  HIPCHK(c, hipGetLastError());
  // inlet velocity, kept for the step's inlet update
  for (int d = 0; d < 3; ++d) {
    F *dst = (F *)(c->base + c->o_ubc) + (size_t)d * c->Ntot + B.off;
    if (u_bc) {
      hipLaunchKernelGGL((k_from_double<F>), grid, blk, 0, c->stream, stage(c, 5 + d), dst, (F *)nullptr, B.n);
      HIPCHK(c, hipGetLastError());
    } else {
      HIPCHK(c, hipMemsetAsync(dst, 0, nb * sizeof(F), c->stream));
    }
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  // potential
  if (phi) {
    HIPCHK(c, hipMemcpy(stage(c, 0), phi, nb * 8, hipMemcpyHostToDevice));
    hipLaunchKernelGGL((k_from_double<F>), grid, blk, 0, c->stream, stage(c, 0),
                       (F *)(c->base + c->o_phi) + B.off, (F *)nullptr, B.n);
  } else {
    HIPCHK(c, hipMemset(c->base + c->o_phi + B.off * sizeof(F), 0, nb * sizeof(F)));
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

// Runs the statement list with L (lattice), T (population type) and F
// (field type) bound to the context's lattice and storage mode.
#define ELBM_DISPATCH_STORAGE(c, ...)                           \
  switch ((c)->P.storage) {                                     \
    case ELBM_STORAGE_F64: {                                    \
      using T = double;                                         \
      using F = double;                                         \
      __VA_ARGS__;                                              \
    }                                                           \
    case ELBM_STORAGE_F32: {                                    \
      using T = float;                                          \
      using F = double;                                         \
      __VA_ARGS__;                                              \
    }                                                           \
    default: {                                                  \
      using T = float;                                          \
      using F = float;                                          \
      __VA_ARGS__;                                              \
    }                                                           \
  }
#define ELBM_DISPATCH(c, ...)                                   \
  if ((c)->P.lattice == ELBM_LATTICE_D2Q9) {                    \
    using Lat = D2Q9;                                             \
    ELBM_DISPATCH_STORAGE(c, __VA_ARGS__)                       \
  } else {                                                      \
    using Lat = D3Q19;                                            \
    ELBM_DISPATCH_STORAGE(c, __VA_ARGS__)                       \
  }

// ---- device scratch of the allocation-free entry point (elbm_mlp_grad_noalloc)
// The gradient kernel's block partials live in a file-scope device array
// instead of the arena: each GPU the library runs on holds one copy, at its
// own address, until the process ends.  Host code never passes the array's
// name to a kernel (in host code it is a stand-in, not a device address): the
// address comes from hipGetSymbolAddress, taken once per device with that
// device current and kept in g_scratch_ptr.  Every call rewrites all of it
// (each of the MLP_GGRID blocks stores all its MLP_GRAD_SLOTS partials), so
// nothing needs clearing; calls that overlap on one GPU race for it.
constexpr size_t NOALLOC_SCRATCH_FLOATS = (size_t)MLP_GGRID * MLP_GRAD_SLOTS;  // 549 KB
static __device__ __align__(256) float scratch[NOALLOC_SCRATCH_FLOATS];
constexpr int NOALLOC_MAX_DEVICES = 64;
static void *g_scratch_ptr[NOALLOC_MAX_DEVICES];
static std::mutex g_scratch_mu;

elbm_status scratch_address(elbm_ctx *c, float **out) {
  const int dev = c->device;
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(c, ELBM_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = 0;
    HIPCHK(c, hipGetDevice(&cur));
    if (cur != dev) HIPCHK(c, hipSetDevice(dev));
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p)
      return fail(c, ELBM_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = (float *)g_scratch_ptr[dev];
  return ELBM_OK;
}

}  // namespace

extern "C" {

uint32_t elbm_abi_version(void) { return ELBM_ABI_VERSION; }

elbm_status elbm_create(const elbm_params *P, const elbm_box *boxes, int32_t nboxes, elbm_ctx **out) {
  if (!out) return ELBM_EINVAL;
  *out = nullptr;
  if (!P || !boxes || nboxes <= 0) return ELBM_EINVAL;
  if (P->ncomp < 1 || P->ncomp > 2) return ELBM_EINVAL;
  if (P->storage != ELBM_STORAGE_F64 && P->storage != ELBM_STORAGE_F32 && P->storage != ELBM_STORAGE_F32_ALL)
    return ELBM_EINVAL;
  if (P->sor_sweeps < 0 || P->newton_max < 1 || P->newton_max > 1000) return ELBM_EINVAL;
  if (!(P->sor_tol >= 0.0) || P->sor_check_every < 0) return ELBM_EINVAL;
  if (P->strict < 0 || P->strict > (ELBM_STRICT_NEGPOP | ELBM_STRICT_ALPHA)) return ELBM_EINVAL;
  if (P->alpha_iter != ELBM_ITER_NEWTON && P->alpha_iter != ELBM_ITER_HALLEY) return ELBM_EINVAL;
  if (P->lattice != ELBM_LATTICE_D3Q19 && P->lattice != ELBM_LATTICE_D2Q9) return ELBM_EINVAL;
  const bool two_d = P->lattice == ELBM_LATTICE_D2Q9;
  if (two_d && P->alpha_guess == ELBM_GUESS_MLP) return ELBM_EINVAL;  // the network reads 19 ratios
  if (P->inlet_mode < ELBM_INLET_NEIGHBOUR || P->inlet_mode > ELBM_INLET_ADAPTIVE_Z) return ELBM_EINVAL;
  if (two_d && P->inlet_mode == ELBM_INLET_ADAPTIVE_Z) return ELBM_EINVAL;  // one x-y plane
  if (P->charge_model != ELBM_CHARGE_CONSERVING && P->charge_model != ELBM_CHARGE_GENERATOR) return ELBM_EINVAL;
  if (!(P->w_theta > 0.0) || !(P->K_d > 0.0) || !(P->nu0 > 0.0) || !(P->newton_rtol > 0.0)) return ELBM_EINVAL;
  if (P->carreau && !(P->nu_inf > 0.0 && P->lam >= 0.0)) return ELBM_EINVAL;
  if (P->alpha_guess != ELBM_GUESS_STANDARD && P->alpha_guess != ELBM_GUESS_SERIES &&
      P->alpha_guess != ELBM_GUESS_MLP)
    return ELBM_EINVAL;
  elbm_ctx *c = new (std::nothrow) elbm_ctx();
  if (!c) return ELBM_ENOMEM;
  c->P = *P;
  c->Q = two_d ? D2Q9::Q : D3Q19::Q;
  c->esz_pop = P->storage == ELBM_STORAGE_F64 ? 8 : 4;
  c->esz_fld = P->storage == ELBM_STORAGE_F32_ALL ? 4 : 8;
  int64_t off = 0;
  int blk0 = 0;
  for (int b = 0; b < nboxes; ++b) {
    const elbm_box &x = boxes[b];
    if (x.nx < 2 || x.ny < 2 || (two_d ? (x.nz != 1 || x.periodic[2]) : x.nz < 2)) { delete c; return ELBM_EINVAL; }
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
    d.rnx = 1.0 / x.nx; d.rny = 1.0 / x.ny;
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
  c->sor_pairs = true;
  for (const auto &x : c->boxes)
    if ((x.nx & 1) || (int64_t)x.nx * x.ny * x.nz < ((int64_t)1 << 20)) c->sor_pairs = false;
  {
    int nxmax = 0;
    for (const auto &x : c->boxes) nxmax = std::max(nxmax, x.nx);
    const int lmax = BLK + 2 * (nxmax + 1);
    const size_t bytes = (size_t)(two_d ? 1 : 3) * lmax * c->esz_fld;
    if (bytes <= 32768) {  // at most 32 KB per block: the stencils keep their occupancy
      c->slab_lmax = lmax;
      c->slab_bytes = bytes;
    }
  }
  for (int s = 1; s < NTILE_SHAPES; ++s) {
    int t0 = 0;
    for (int b = 0; b < nboxes; ++b) {
      const elbm_box &x = boxes[b];
      const int ntx = (x.nx + tile_dim(s, 0) - 1) / tile_dim(s, 0), nty = (x.ny + tile_dim(s, 1) - 1) / tile_dim(s, 1),
                ntz = (x.nz + tile_dim(s, 2) - 1) / tile_dim(s, 2);
      c->box_tiles[s].push_back(int4{t0, ntx, nty, ntz});
      const int nt = ntx * nty * ntz;
      for (int i = 0; i < nt; ++i) c->tile_box[s].push_back(b);
      t0 += nt;
    }
    c->ntiles[s] = t0;
  }
  const int C = P->ncomp;
  const int64_t N = c->Ntot;
  const size_t e = c->esz_fld, ep = c->esz_pop;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
  c->o_fa = take((size_t)C * c->Q * N * ep);
  c->o_fb = take((size_t)C * c->Q * N * ep);
  c->o_rho = take((size_t)C * N * e);
  c->o_psi = take((size_t)C * N * e);
  c->o_grad = take(4 * (size_t)N * e);
  c->o_bulk = take((size_t)N * e);
  c->o_surf = take((size_t)N * e);
  c->o_q = take((size_t)N * e);
  c->o_phi = take((size_t)N * e);
  c->o_rhs = take((size_t)N * e);
  c->o_e2 = take((size_t)N * e);
  c->o_recu = take(3 * (size_t)N * e);
  c->o_ubc = take(3 * (size_t)N * e);
  c->o_ab = take((size_t)C * N * 8);
  c->o_nbm = take((size_t)N * 4);
  c->o_reca = take((size_t)C * N * 8);
  c->o_reci = take((size_t)C * N * 4);
  c->o_type = take((size_t)N);
  c->o_stage = take(9 * (size_t)c->maxN * 8);
  c->o_boxes = take(sizeof(BoxDev) * nboxes);
  c->o_bb = take(sizeof(int32_t) * c->nblocks);
  c->o_part = take(sizeof(double) * 4 * (size_t)c->nblocks);
  c->o_rpart = take(sizeof(double) * 2 * (size_t)c->nblocks);
  c->o_fpart = take(sizeof(double) * 3 * (size_t)c->nblocks);
  c->o_npart = take(sizeof(double) * 2 * (size_t)c->nblocks);
  c->o_scal = take(sizeof(double) * NSCAL * nboxes);
  c->o_cnt = take(sizeof(unsigned long long) * NCNT * nboxes);
  c->o_err = take(sizeof(uint32_t) * 4);
  c->o_mp = take(sizeof(float) * MLP_NPARAM);
  c->o_mm = take(sizeof(float) * MLP_NPARAM);
  c->o_mv = take(sizeof(float) * MLP_NPARAM);
  c->o_mw1 = take(2 * 32 * 32);
  c->o_mw2 = take(2 * 32 * 32);
  c->o_mw2t = take(2 * 32 * 32);
  c->o_mgrad = take(sizeof(float) * (MLP_NPARAM + 1));
  c->o_mpart = take(sizeof(float) * MLP_GGRID * MLP_GRAD_SLOTS);
  c->o_mloss = take(sizeof(float) * MLP_MAX_STEPS);
  for (int s = 1; s < NTILE_SHAPES; ++s) {
    c->o_tbox[s] = take(sizeof(int32_t) * c->tile_box[s].size());
    c->o_btiles[s] = take(sizeof(int4) * c->box_tiles[s].size());
  }
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
  c->drop_graphs();
  HIPCHK(c, hipGetDevice(&c->device));
  c->base = (char *)arena;
  c->stream = (hipStream_t)stream;
  if (!c->aux) {  // default priority, like the caller's stream
    HIPCHK(c, hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
    HIPCHK(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    HIPCHK(c, hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
  }
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
  // the collision's tile tables live past the cleared region's start: upload after the clear
  for (int s = 1; s < NTILE_SHAPES; ++s) {
    HIPCHK(c, hipMemcpy(c->base + c->o_tbox[s], c->tile_box[s].data(), sizeof(int32_t) * c->tile_box[s].size(),
                        hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->base + c->o_btiles[s], c->box_tiles[s].data(), sizeof(int4) * c->box_tiles[s].size(),
                        hipMemcpyHostToDevice));
  }

  c->bound = true;
  return ELBM_OK;
}

elbm_status elbm_set_box(elbm_ctx *c, int32_t box, const uint8_t *type, const double *rho, const double *u,
                         const double *phi, const double *u_bc, const double *xi, double jitter) {
  elbm_status st = check_box_arg(c, box);
  if (st) return st;
  if (!type || !rho) return fail(c, ELBM_EINVAL, "node_type and rho are required");
  // steps in flight read the box table and may run a captured graph: finish
  // them before the graphs are dropped and the box record is rewritten
  HIPCHK(c, hipStreamSynchronize(c->stream));
  BoxDev &B = c->bdev[box];
  int64_t nu = 0;
  bool dir = false;
  for (int i = 0; i < B.n; ++i) {
    if (type[i] > 15) return fail(c, ELBM_EINVAL, "node type byte out of range");
    if ((type[i] & B_NOZZLE) && (type[i] & 3) != K_FLUID) return fail(c, ELBM_EINVAL, "NOZZLE bit on a non-fluid node");
    if (type[i] & B_DIRICHLET) dir = true; else ++nu;
  }
  B.has_dirichlet = dir ? 1 : 0;
  B.n_unknown = (int32_t)nu;
  c->drop_graphs();  // the gauge launches depend on the Dirichlet flags
  c->any_gauge = false;
  for (auto &d : c->bdev) if (!d.has_dirichlet) c->any_gauge = true;
  HIPCHK(c, hipMemcpy(c->base + c->o_boxes + sizeof(BoxDev) * box, &B, sizeof(BoxDev), hipMemcpyHostToDevice));
  ELBM_DISPATCH(c, return set_box_impl<Lat, T, F>(c, box, type, rho, u, phi, u_bc, xi, jitter))
}

elbm_status elbm_step(elbm_ctx *c, int32_t nsteps, int32_t record) {
  if (!c) return ELBM_EINVAL;
  if (!c->bound) return fail(c, ELBM_ESTATE, "context is not bound to an arena");
  if (nsteps < 0) return fail(c, ELBM_EINVAL, "nsteps must be >= 0");
  if (nsteps == 0) return ELBM_OK;
  if (c->P.ncomp == 2) {
    ELBM_DISPATCH(c, return launch_steps<Lat, T, F, 2>(c, nsteps, record))
  }
  ELBM_DISPATCH(c, return launch_steps<Lat, T, F, 1>(c, nsteps, record))
}

elbm_status elbm_set_graphs(elbm_ctx *c, int32_t enable) {
  if (!c) return ELBM_EINVAL;
  if (c->bound) HIPCHK(c, hipStreamSynchronize(c->stream));
  c->use_graphs = enable != 0;
  if (!c->use_graphs) c->drop_graphs();
  return ELBM_OK;
}

elbm_status elbm_set_launch(elbm_ctx *c, const elbm_launch *l) {
  if (!c || !l) return ELBM_EINVAL;
  if (l->xcd_remap != 0 && l->xcd_remap != 1) return fail(c, ELBM_EINVAL, "xcd_remap must be 0 or 1");
  if (l->graph_steps < 2 || l->graph_steps > 64 || (l->graph_steps & 1))
    return fail(c, ELBM_EINVAL, "graph_steps must be even, 2..64");
  if (l->tile < 0 || l->tile >= NTILE_SHAPES) return fail(c, ELBM_EINVAL, "tile must be 0..3");
  if (l->sweep_priority != 0 && l->sweep_priority != 1) return fail(c, ELBM_EINVAL, "sweep_priority must be 0 or 1");
  if (l->stencil_lds != 0 && l->stencil_lds != 1) return fail(c, ELBM_EINVAL, "stencil_lds must be 0 or 1");
  if (l->stencil_lds && !c->slab_lmax)
    return fail(c, ELBM_EINVAL, "stencil_lds: the LDS slabs of the widest box exceed 32 KB per block");
  if (c->bound) HIPCHK(c, hipStreamSynchronize(c->stream));
  c->remap = l->xcd_remap;
  c->graph_steps = l->graph_steps;
  c->tile = l->tile;
  c->prio = l->sweep_priority;
  c->slabs = l->stencil_lds != 0;
  c->drop_graphs();  // kernel arguments and step counts are baked into the graphs
  return ELBM_OK;
}

elbm_status elbm_get_launch(const elbm_ctx *c, elbm_launch *l) {
  if (!c || !l) return ELBM_EINVAL;
  l->xcd_remap = c->remap;
  l->graph_steps = c->graph_steps;
  l->tile = c->tile;
  l->sweep_priority = c->prio;
  l->stencil_lds = c->slabs ? 1 : 0;
  return ELBM_OK;
}

// Times one launch mapping over `trial` steps (after the steps that capture
// its graph); ms per step into *ms.
static elbm_status time_launch(elbm_ctx *c, const elbm_launch &l, int trial, hipEvent_t e0, hipEvent_t e1,
                               double *ms) {
  elbm_status st = elbm_set_launch(c, &l);
  if (!st) st = elbm_step(c, l.graph_steps, 0);
  if (st) return st;
  if (hipEventRecord(e0, c->stream) != hipSuccess) return fail(c, ELBM_EHIP, "hipEventRecord");
  st = elbm_step(c, trial, 0);
  if (st) return st;
  float t = 0.f;
  if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
      hipEventElapsedTime(&t, e0, e1) != hipSuccess)
    return fail(c, ELBM_EHIP, "autotune timing");
  *ms = t / trial;
  return ELBM_OK;
}

elbm_status elbm_autotune(elbm_ctx *c, int32_t steps_per_trial, elbm_launch *best, double *ms_per_step) {
  if (!c) return ELBM_EINVAL;
  if (!c->bound) return fail(c, ELBM_ESTATE, "context is not bound to an arena");
  if (c->timing) return fail(c, ELBM_ESTATE, "autotune with phase timing on");
  if (steps_per_trial < 1) return fail(c, ELBM_EINVAL, "steps_per_trial must be >= 1");
  const int trial = (steps_per_trial + 15) / 16 * 16;  // whole replays of every candidate
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  const elbm_launch keep{c->remap, c->graph_steps, c->tile, c->prio, c->slabs ? 1 : 0};
  elbm_launch cur{0, 2, 0, 0, 0};  // the stencils' LDS slabs are not among the candidates
  elbm_status st = ELBM_OK;
  // four passes, each fixing one knob with the winners of the earlier ones:
  // tile shape (4), XCD order (2), field-chain priority (2), graph length
  // (3; last, so that every earlier trial captures 2 steps); within a pass two
  // rounds, forward then reverse order, and a candidate's time is the mean of
  // its two: a state that drifts linearly during the trials (an initial
  // transient) then favours no candidate
  static const int kSteps[3] = {2, 4, 8};
  int slot = 0;
  for (int pass = 0; pass < 4 && !st; ++pass) {
    const int n = pass == 0 ? NTILE_SHAPES : pass == 3 ? 3 : 2;
    double per[NTILE_SHAPES];
    for (int k = 0; k < n; ++k) per[k] = 0.0;
    for (int t = 0; t < 2 * n && !st; ++t) {
      const int k = t < n ? t : 2 * n - 1 - t;
      elbm_launch l = cur;
      if (pass == 0) l.tile = k;
      else if (pass == 1) l.xcd_remap = k;
      else if (pass == 2) l.sweep_priority = k;
      else l.graph_steps = kSteps[k];
      double ms = 0.0;
      st = time_launch(c, l, trial, e0, e1, &ms);
      if (!st) per[k] += 0.5 * ms;
    }
    if (st) break;
    int kb = 0;
    for (int k = 0; k < n; ++k) {
      if (ms_per_step) ms_per_step[slot + k] = per[k];
      if (per[k] < per[kb]) kb = k;
    }
    slot += n;
    if (pass == 0) cur.tile = kb;
    else if (pass == 1) cur.xcd_remap = kb;
    else if (pass == 2) cur.sweep_priority = kb;
    else cur.graph_steps = kSteps[kb];
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) {
    (void)elbm_set_launch(c, &keep);
    return st;
  }
  st = elbm_set_launch(c, &cur);
  if (!st && best) *best = cur;
  return st;
}

elbm_status elbm_sync(elbm_ctx *c) {
  if (!c) return ELBM_EINVAL;
  if (!c->bound) return fail(c, ELBM_ESTATE, "context is not bound to an arena");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  uint32_t e = 0;
  HIPCHK(c, hipMemcpy(&e, c->base + c->o_err, sizeof(e), hipMemcpyDeviceToHost));
  if (e & ERR_NONFINITE) return fail(c, ELBM_ENONFINITE, "a post-collision population became non-finite");
  if (e & ERR_NEGPOP) return fail(c, ELBM_ENEGPOP, "a post-collision population became negative (strict)");
  if (e & ERR_SOR) return fail(c, ELBM_ENOCONV, "a Poisson solve ended above sor_tol");
  if (e & ERR_ALPHA) return fail(c, ELBM_ENOCONV, "an alpha solve fell back: no root or no convergence (strict)");
  return ELBM_OK;
}

elbm_status elbm_read_moments(elbm_ctx *c, int32_t box, double *rho, double *u) {
  elbm_status st = check_box_arg(c, box);
  if (st) return st;
  if (rho) {
    ELBM_DISPATCH(c, st = read_planes<F>(c, box, c->o_rho, c->P.ncomp, rho); break)
    if (st) return st;
  }
  if (u) {
    ELBM_DISPATCH(c, st = read_planes<F>(c, box, c->o_recu, 3, u); break)
  }
  return st;
}

elbm_status elbm_read_potential(elbm_ctx *c, int32_t box, double *phi) {
  elbm_status st = check_box_arg(c, box);
  if (st) return st;
  if (!phi) return fail(c, ELBM_EINVAL, "phi is NULL");
  ELBM_DISPATCH(c, return read_planes<F>(c, box, c->o_phi, 1, phi))
}

elbm_status elbm_read_charge(elbm_ctx *c, int32_t box, double *q) {
  elbm_status st = check_box_arg(c, box);
  if (st) return st;
  if (!q) return fail(c, ELBM_EINVAL, "q is NULL");
  ELBM_DISPATCH(c, return read_planes<F>(c, box, c->o_q, 1, q))
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
  const int np = c->P.ncomp * c->Q;
  ELBM_DISPATCH(c, return read_planes<T>(c, box, cur_pop_off(c), np, f))
}

elbm_status elbm_set_populations(elbm_ctx *c, int32_t box, const double *f) {
  elbm_status st = check_box_arg(c, box);
  if (st) return st;
  if (!f) return fail(c, ELBM_EINVAL, "f is NULL");
  const int np = c->P.ncomp * c->Q;
  const size_t other = c->parity ? c->o_fa : c->o_fb;
  ELBM_DISPATCH(c, return write_planes<T>(c, box, cur_pop_off(c), other, np, f))
}

elbm_status elbm_set_potential(elbm_ctx *c, int32_t box, const double *phi) {
  elbm_status st = check_box_arg(c, box);
  if (st) return st;
  if (!phi) return fail(c, ELBM_EINVAL, "phi is NULL");
  ELBM_DISPATCH(c, return write_planes<F>(c, box, c->o_phi, 0, 1, phi))
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
  ELBM_DISPATCH(c, {
    Ptrs<T, F> a = make_ptrs<T, F>(c);
    if (c->P.ncomp == 2) hipLaunchKernelGGL((k_diag<Lat, T, F, 2>), grid, blk, 0, c->stream, a, box, dst);
    else hipLaunchKernelGGL((k_diag<Lat, T, F, 1>), grid, blk, 0, c->stream, a, box, dst);
  } break)
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  // block partials in block order (a fixed-order sum, reproducible)
  std::vector<double> part((size_t)nblk * DIAG_W);
  HIPCHK(c, hipMemcpy(part.data(), dst, part.size() * 8, hipMemcpyDeviceToHost));
  double asum = 0.0, acnt = 0.0, amin = INFINITY, amax = -INFINITY;
  for (int i = 0; i < nblk; ++i) {
    const double *v = part.data() + (size_t)i * DIAG_W;
    out->mass[0] += v[0];
    out->mass[1] += v[1];
    for (int d = 0; d < 3; ++d) out->momentum[d] += v[2 + d];
    asum += v[5];
    acnt += v[6];
    amin = fmin(amin, -v[7]);
    amax = fmax(amax, v[8]);
  }
  out->alpha_min = acnt > 0.0 ? amin : 0.0;
  out->alpha_max = acnt > 0.0 ? amax : 0.0;
  out->alpha_mean = acnt > 0.0 ? asum / acnt : 0.0;
  // electric force of the last recorded step: the box's block partials in order
  std::vector<double> fp((size_t)B.nblocks * 3);
  HIPCHK(c, hipMemcpy(fp.data(), (double *)(c->base + c->o_fpart) + (size_t)B.first_block * 3, fp.size() * 8,
                      hipMemcpyDeviceToHost));
  for (int i = 0; i < B.nblocks; ++i)
    for (int d = 0; d < 3; ++d) out->sum_Fel[d] += fp[(size_t)i * 3 + d];
  double sc[NSCAL];
  HIPCHK(c, hipMemcpy(sc, c->base + c->o_scal + sizeof(double) * NSCAL * box, sizeof(sc), hipMemcpyDeviceToHost));
  out->sor_residual = sc[4];
  out->sor_scale = sc[5];
  out->sor_sweeps = (int32_t)sc[6];
  out->inlet_ubar = sc[8];
  unsigned long long cn[NCNT];
  HIPCHK(c, hipMemcpy(cn, c->base + c->o_cnt + sizeof(unsigned long long) * NCNT * box, sizeof(cn), hipMemcpyDeviceToHost));
  out->n_fallback = (int64_t)cn[0];
  out->n_negative = (int64_t)cn[2];
  out->n_collisions = (int64_t)cn[4];
  out->n_sor_noconv = (int64_t)cn[5];
  const int64_t solved = (int64_t)cn[4] - (int64_t)cn[0];
  out->mean_newton_iters = solved > 0 ? (double)cn[1] / (double)solved : 0.0;
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

elbm_status elbm_mlp_set_weights(elbm_ctx *c, const float *w, int64_t n) {
  if (!c) return ELBM_EINVAL;
  if (!c->bound) return fail(c, ELBM_ESTATE, "context is not bound to an arena");
  if (!w || n != MLP_NPARAM) return fail(c, ELBM_EINVAL, "weights: need 1761 floats");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(c->base + c->o_mp, w, sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemset(c->base + c->o_mm, 0, sizeof(float) * MLP_NPARAM));
  HIPCHK(c, hipMemset(c->base + c->o_mv, 0, sizeof(float) * MLP_NPARAM));
  c->adam_t = 0;
  hipLaunchKernelGGL(k_mlp_refresh, dim3(1), dim3(BLK), 0, c->stream, (const float *)(c->base + c->o_mp),
                     (__bf16 *)(c->base + c->o_mw1), (__bf16 *)(c->base + c->o_mw2),
                     (__bf16 *)(c->base + c->o_mw2t));
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return ELBM_OK;
}

elbm_status elbm_mlp_get_weights(elbm_ctx *c, float *w, int64_t n) {
  if (!c) return ELBM_EINVAL;
  if (!c->bound) return fail(c, ELBM_ESTATE, "context is not bound to an arena");
  if (!w || n != MLP_NPARAM) return fail(c, ELBM_EINVAL, "weights: need 1761 floats");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(w, c->base + c->o_mp, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost));
  return ELBM_OK;
}

elbm_status elbm_mlp_forward(elbm_ctx *c, const void *dX, void *dY, int64_t M) {
  if (!c) return ELBM_EINVAL;
  if (!c->bound) return fail(c, ELBM_ESTATE, "context is not bound to an arena");
  if (!dX || !dY || M < 0) return fail(c, ELBM_EINVAL, "mlp_forward: bad arguments");
  if (M == 0) return ELBM_OK;
  const int64_t nb = (M + BLK - 1) / BLK;
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)(nb < 4096 ? nb : 4096)), dim3(BLK), 0, c->stream, make_mlp(c),
                     (const float *)dX, (float *)dY, M);
  HIPCHK(c, hipGetLastError());
  return ELBM_OK;
}

elbm_status elbm_mlp_grad(elbm_ctx *c, const void *dX, const void *dT, int64_t M, float *grad, float *loss) {
  if (!c) return ELBM_EINVAL;
  if (!c->bound) return fail(c, ELBM_ESTATE, "context is not bound to an arena");
  if (!dX || !dT || M <= 0) return fail(c, ELBM_EINVAL, "mlp_grad: bad arguments");
  float *part = (float *)(c->base + c->o_mpart), *g = (float *)(c->base + c->o_mgrad);
  hipLaunchKernelGGL(k_mlp_grad, dim3(MLP_GGRID), dim3(MLP_GBLK), 0, c->stream, make_mlp(c), (const float *)dX,
                     (const float *)dT, (int64_t)0, M, 1.0f / (float)M, part);
  hipLaunchKernelGGL(k_mlp_sum, dim3(1), dim3(BLK), 0, c->stream, (const float *)part, MLP_GGRID, g, (float *)nullptr);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (grad) HIPCHK(c, hipMemcpy(grad, g, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost));
  if (loss) HIPCHK(c, hipMemcpy(loss, g + MLP_NPARAM, sizeof(float), hipMemcpyDeviceToHost));
  return ELBM_OK;
}

elbm_status elbm_mlp_grad_noalloc(elbm_ctx *c, const void *dX, const void *dT, int64_t M, void *dGrad) {
  if (!c) return ELBM_EINVAL;
  if (!c->bound) return fail(c, ELBM_ESTATE, "context is not bound to an arena");
  if (!dX || !dT || !dGrad || M <= 0) return fail(c, ELBM_EINVAL, "mlp_grad_noalloc: bad arguments");
  // the scratch holds MLP_GGRID block partials whatever M is: no size of the
  // call can exceed it
  static_assert(NOALLOC_SCRATCH_FLOATS >= (size_t)MLP_GGRID * MLP_GRAD_SLOTS, "scratch too small for the grid");
  float *part = nullptr;
  elbm_status st = scratch_address(c, &part);
  if (st) return st;
  hipLaunchKernelGGL(k_mlp_grad, dim3(MLP_GGRID), dim3(MLP_GBLK), 0, c->stream, make_mlp(c), (const float *)dX,
                     (const float *)dT, (int64_t)0, M, 1.0f / (float)M, part);
  hipLaunchKernelGGL(k_mlp_sum, dim3(1), dim3(BLK), 0, c->stream, (const float *)part, MLP_GGRID, (float *)dGrad,
                     (float *)nullptr);
  HIPCHK(c, hipGetLastError());
  return ELBM_OK;
}

elbm_status elbm_mlp_train(elbm_ctx *c, const void *dX, const void *dT, int64_t M, int32_t batch, int32_t steps,
                           float lr, float *losses) {
  if (!c) return ELBM_EINVAL;
  if (!c->bound) return fail(c, ELBM_ESTATE, "context is not bound to an arena");
  if (!dX || !dT || M <= 0 || batch <= 0 || steps < 0 || steps > MLP_MAX_STEPS || !(lr > 0.0f))
    return fail(c, ELBM_EINVAL, "mlp_train: bad arguments");
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  float *part = (float *)(c->base + c->o_mpart), *g = (float *)(c->base + c->o_mgrad);
  float *lbuf = (float *)(c->base + c->o_mloss);
  int64_t start = 0;
  for (int i = 0; i < steps; ++i) {
    if (start >= M) start = 0;
    const int64_t B = (start + batch <= M) ? batch : M - start;
    hipLaunchKernelGGL(k_mlp_grad, dim3(MLP_GGRID), dim3(MLP_GBLK), 0, c->stream, make_mlp(c), (const float *)dX,
                       (const float *)dT, start, B, 1.0f / (float)B, part);
    hipLaunchKernelGGL(k_mlp_sum, dim3(1), dim3(BLK), 0, c->stream, (const float *)part, MLP_GGRID, g, lbuf + i);
    c->adam_t += 1;
    const float bc1 = 1.0f - powf(b1, (float)c->adam_t), bc2 = 1.0f - powf(b2, (float)c->adam_t);
    hipLaunchKernelGGL(k_mlp_adam, dim3(1), dim3(BLK), 0, c->stream, (float *)(c->base + c->o_mp),
                       (float *)(c->base + c->o_mm), (float *)(c->base + c->o_mv), (const float *)g, lr, b1, b2, eps,
                       bc1, bc2);
    hipLaunchKernelGGL(k_mlp_refresh, dim3(1), dim3(BLK), 0, c->stream, (const float *)(c->base + c->o_mp),
                       (__bf16 *)(c->base + c->o_mw1), (__bf16 *)(c->base + c->o_mw2),
                       (__bf16 *)(c->base + c->o_mw2t));
    start += B;
  }
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (losses && steps > 0) HIPCHK(c, hipMemcpy(losses, lbuf, sizeof(float) * steps, hipMemcpyDeviceToHost));
  return ELBM_OK;
}

elbm_status elbm_alpha_samples(elbm_ctx *c, int32_t box, void *dFeat, void *dTarget, void *dScale,
                               void *dValid) {
  elbm_status st = check_box_arg(c, box);
  if (st) return st;
  if (!dFeat || !dTarget || !dScale || !dValid) return fail(c, ELBM_EINVAL, "alpha_samples: NULL output");
  if (c->P.lattice != ELBM_LATTICE_D3Q19) return fail(c, ELBM_EINVAL, "alpha_samples: the learned starter is D3Q19");
  const Model M = make_model(c->P);
  const dim3 grid(c->nblocks), blk(BLK);
  if (c->P.ncomp == 2) {
    ELBM_DISPATCH(c, {
      hipLaunchKernelGGL((k_alpha_samples<T, F, 2>), grid, blk, 0, c->stream, make_ptrs<T, F>(c), M, box,
                         (float *)dFeat, (float *)dTarget, (float *)dScale, (int32_t *)dValid);
    } break)
  } else {
    ELBM_DISPATCH(c, {
      hipLaunchKernelGGL((k_alpha_samples<T, F, 1>), grid, blk, 0, c->stream, make_ptrs<T, F>(c), M, box,
                         (float *)dFeat, (float *)dTarget, (float *)dScale, (int32_t *)dValid);
    } break)
  }
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return ELBM_OK;
}

const char *elbm_last_error(const elbm_ctx *c) {
  if (!c) return "null context";
  return c->err.c_str();
}

void elbm_destroy(elbm_ctx *c) { delete c; }

}  // extern "C"
