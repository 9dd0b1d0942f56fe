/*
 * elbm.h -- C ABI of the MI355X (gfx950) library for the per-time-step
 * lattice update of the entropic lattice Boltzmann model for charged
 * leaky-dielectric multiphase fluids (Lauricella et al., arXiv:1612.05404).
 *
 * One step (Sec. II.C, "Summary of the model") on a D3Q19 lattice with one
 * or two Shan-Chen components:
 *   streaming of Eq. lattice-b by pulling, halfway bounce-back at walls;
 *   free charge from Eq. surface-q2 (conserving) or Eq. surface-q3
 *   (generator-connected), with the curvature of Eq. surface-curvature;
 *   Poisson equation div(eps grad phi) = -q (Sec. II, Gauss law) by red-black
 *   SOR with a neutralising uniform charge;
 *   electric force Eq. force_el2; Shan-Chen force Eq. sc;
 *   entropic alpha from Eqs. entropic and H (FP64 Newton per node);
 *   Carreau viscosity, Eqs. strain2 and carreau, and beta from Eq. beta;
 *   collision Eq. lattice-b with the exact-difference source Eq. add.
 *
 * Conventions.
 *  - Every call returns an elbm_status (0 = ok, < 0 = error); nothing throws
 *    or aborts across the ABI.  elbm_last_error() gives a message.
 *  - Host arrays are caller-owned, FP64, C order with x fastest:
 *    a scalar field is [nz][ny][nx], a component field [C][nz][ny][nx],
 *    a vector field [3][nz][ny][nx], populations [C][19][nz][ny][nx].
 *  - D3Q19 order: p = 0 rest; 1..6 = +x, -x, +y, -y, +z, -z;
 *    7..18 = (+1,+1,0), (-1,-1,0), (+1,-1,0), (-1,+1,0), (+1,0,+1), (-1,0,-1),
 *    (+1,0,-1), (-1,0,+1), (0,+1,+1), (0,-1,-1), (0,+1,-1), (0,-1,+1).
 *    Opposite directions sit at adjacent (odd, even) indices.
 *  - Node-type byte: bits 0-1 = 0 fluid, 1 solid wall, 2 inlet, 3 outlet;
 *    bit 2 = potential fixed (Dirichlet node of the Poisson problem).
 *  - Device memory: the caller allocates one arena of elbm_required_bytes()
 *    bytes and passes it with a HIP stream to elbm_bind().  The library never
 *    allocates device memory; it enqueues all work on that stream.  The arena
 *    and the stream must outlive the context.  A context is not thread-safe.
 */
#ifndef ELBM_H
#define ELBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ELBM_ABI_VERSION 7u  /* 2: fluid-wall coupling matrix Gw[2][2]; alpha phase in the timing;
                                 3: sweep_priority in elbm_launch;
                                 4: Poisson stop rule and residual, strict error flags, Halley
                                    iteration, electric force and solver fields in elbm_diag;
                                 5: the lattice (D3Q19 or the paper's D2Q9) in elbm_params;
                                 6: the adaptive jet inlet (inlet_mode, NOZZLE nodes, the
                                    measured mean velocity in elbm_diag);
                                 7: stencil_lds in elbm_launch */

typedef struct elbm_ctx elbm_ctx;

typedef enum {
    ELBM_OK = 0,
    ELBM_EINVAL = -1,      /* bad argument: nothing was enqueued            */
    ELBM_ENOMEM = -2,      /* arena too small or host allocation failed     */
    ELBM_EHIP = -3,        /* a HIP runtime call failed                     */
    ELBM_ENONFINITE = -4,  /* a post-collision population became non-finite */
    ELBM_ENEGPOP = -5,     /* a post-collision population became negative
                              (only with ELBM_STRICT_NEGPOP)                */
    ELBM_ENOCONV = -6,     /* a Poisson solve ended above its tolerance, or
                              (with ELBM_STRICT_ALPHA) an alpha solve fell
                              back                                          */
    ELBM_ESTATE = -7       /* call out of order (e.g. step before bind)     */
} elbm_status;

/* elbm_params.strict: device conditions that, besides non-finite
 * populations (always), set the sticky error word that elbm_sync reports.
 * Without them the conditions are only counted (elbm_diag). */
enum { ELBM_STRICT_NEGPOP = 1, ELBM_STRICT_ALPHA = 2 };

/* Lattice (Sec. II, Eq. lattice-b): D3Q19, or D2Q9, the paper's own 2-D
 * lattice (p = 0 rest; 1..4 = +x, -x, +y, -y; 5..8 = (+1,+1), (-1,-1),
 * (+1,-1), (-1,+1); weights 4/9, 1/9, 1/36).  A D2Q9 box is one x-y plane:
 * nz = 1 and bounded in z (the Poisson problem then has no z faces);
 * populations are [C][9][N]. */
enum { ELBM_LATTICE_D3Q19 = 0, ELBM_LATTICE_D2Q9 = 1 };

/* Node type byte (elbm_set_box): bits 0-1 the kind, FLUID 0, SOLID 1 (halfway
 * bounce-back), INLET 2, OUTLET 3; bit 2 DIRICHLET (the potential is held at
 * its initial value); bit 3 NOZZLE, on fluid nodes only: the node enters the
 * mean velocity that the adaptive inlet measures. */
enum { ELBM_NODE_FLUID = 0, ELBM_NODE_SOLID = 1, ELBM_NODE_INLET = 2, ELBM_NODE_OUTLET = 3,
       ELBM_NODE_DIRICHLET = 4, ELBM_NODE_NOZZLE = 8 };

/* Inlet nodes (the jet set-up of Sec. III.B).  NEIGHBOUR: each step an inlet
 * node is reset to f_eq(rho_nb, u_bc) per component, rho_nb the w-weighted
 * mean density of its fluid neighbours (rho_in when it has none).
 * ADAPTIVE_X/Y/Z, the paper's inlet: f_eq(rho_in, ubar u_bc), u_bc the
 * velocity profile (its shape; a unit mean gives the measured flow rate) and
 * ubar the mean velocity of the fluid inside the nozzle along that axis,
 * sum_nozzle sum_s j_s / sum_nozzle sum_s rho_s over the NOZZLE nodes, from
 * the same step's streamed moments; inlet nodes start from rest. */
enum { ELBM_INLET_NEIGHBOUR = 0, ELBM_INLET_ADAPTIVE_X = 1, ELBM_INLET_ADAPTIVE_Y = 2,
       ELBM_INLET_ADAPTIVE_Z = 3 };

/* Storage: F64 = FP64 populations and fields; F32 = FP32 populations with
 * FP64 auxiliary fields (densities, psi, charge, potential, |E|^2);
 * F32_ALL = FP32 populations and fields.  Alpha and the collision moments
 * are FP64 in every mode. */
enum { ELBM_STORAGE_F64 = 0, ELBM_STORAGE_F32 = 1, ELBM_STORAGE_F32_ALL = 2 };
enum { ELBM_CHARGE_CONSERVING = 0, ELBM_CHARGE_GENERATOR = 1 };
/* Initial guess of the alpha iteration; every guess is polished to the
 * same stopping rule.  STANDARD: alpha0 = 2 (the BGK value).  SERIES: root of
 * the degree-11 truncation of the entropy balance in powers of alpha (no
 * logarithms), used inside the positivity interval while alpha0 max|x| < 1.2.
 * MLP: the series starter where it is used, the learned starter elsewhere
 * (see elbm_mlp_* below). */
enum { ELBM_GUESS_STANDARD = 0, ELBM_GUESS_MLP = 1, ELBM_GUESS_SERIES = 2 };
/* The iteration itself: NEWTON on the entropy balance g(alpha) = H(f +
 * alpha Delta) - H(f) (Eqs. entropic, H), or HALLEY, which also uses
 * g'' = sum_p Delta_p x_p / (1 + alpha x_p) (no further logarithm). */
enum { ELBM_ITER_NEWTON = 0, ELBM_ITER_HALLEY = 1 };

/* Model constants shared by every box of a context. */
typedef struct {
    int32_t ncomp;            /* 1 (the paper's single fluid) or 2 components       */
    int32_t storage;          /* ELBM_STORAGE_*                                     */
    int32_t carreau;          /* 1: Carreau viscosity (Eq. carreau), 0: nu = nu0     */
    int32_t curvature;        /* 1: surface-charge factor 1 + (K/K_d)^(1/4)          */
    int32_t electrostriction; /* 1: F_el = qE + (eps-1)/2 grad|E|^2, 0: F_el = qE    */
    int32_t charge_model;     /* ELBM_CHARGE_*                                      */
    int32_t sor_sweeps;       /* red-black SOR sweeps per step (>= 0)               */
    int32_t newton_max;       /* max Newton updates for alpha (>= 1)                */
    int32_t alpha_guess;      /* ELBM_GUESS_*                                       */
    int32_t strict;           /* ELBM_STRICT_* mask (0: only non-finite is an error) */
    double G[2][2];           /* Shan-Chen couplings G[s][s'] (Eq. sc)              */
    double Gw[2][2];          /* fluid-wall couplings Gw[s][s'] (Eq. sc, wall sum): a wall
                                 neighbour carries the node's own psi^s'; Gw = G is a
                                 neutral wall                                       */
    double nu0, nu_inf, lam;  /* viscosity (Newtonian: nu0), Carreau nu_inf, lambda */
    double K_d;               /* curvature doubling the surface charge              */
    double rho_th, w_theta;   /* smoothed Heaviside: 0.5(1+tanh((rho-rho_th)/w))    */
    double xi_b, xi_s;        /* generator-connected charge constants (Eq. surface-q3) */
    double newton_rtol;       /* alpha converged when |dH| <= rtol * scale          */
    double rho_in[2];         /* inlet densities: at start, for a neighbour inlet
                                 node without fluid neighbours, and always with an
                                 adaptive inlet                                     */
    double rho_out[2];        /* component densities held at outlet nodes           */
    double sor_tol;           /* > 0: Poisson sweeps stop once the residual
                                 max|sum_f eps_f (phi_nb - phi) - rhs| is at most
                                 sor_tol * max|rhs| (unknown nodes of the box, FP64),
                                 and a solve that ends above it sets ELBM_ENOCONV;
                                 0: exactly sor_sweeps sweeps                      */
    int32_t sor_check_every;  /* with sor_tol > 0: residual checked after every so
                                 many sweeps (0: after the last only)              */
    int32_t alpha_iter;       /* ELBM_ITER_*                                        */
    int32_t lattice;          /* ELBM_LATTICE_* (the learned starter: D3Q19 only)    */
    int32_t inlet_mode;       /* ELBM_INLET_*                                       */
} elbm_params;

/* One lattice box.  Boxes of one context are independent (no exchange). */
typedef struct {
    int32_t nx, ny, nz;       /* >= 2 each (D2Q9: nz = 1); a periodic axis must have
                                 even length                                        */
    int32_t periodic[3];      /* 1 = periodic along x, y, z; 0 = bounded            */
    double E_ext[3];          /* uniform external field                             */
    double Q_b, Q_s;          /* bulk and surface charge (conserving model)         */
    double n_flow;            /* Carreau flow index n                               */
    double sor_omega;         /* SOR over-relaxation factor in (0, 2)               */
} elbm_box;

/* Diagnostics of one box (conservation checks of Sec. II.C: mass per
 * component, momentum, the electric body force; solver statistics). */
typedef struct {
    double mass[2];           /* sum over nodes of sum_p f, per component           */
    double momentum[3];       /* sum over nodes, components and p of c_p f          */
    double alpha_min, alpha_max, alpha_mean;  /* over fluid (node, component) pairs,
                                 last recorded step (device reduction)             */
    double mean_newton_iters; /* alpha updates per (node, component), all steps     */
    int64_t n_fallback;       /* alpha fallbacks (no root / no convergence), all steps */
    int64_t n_negative;       /* negative post-collision populations, all steps     */
    int64_t n_collisions;     /* (node, component) collisions counted, all steps    */
    double sum_Fel[3];        /* sum over fluid nodes of the electric force Eq.
                                 force_el2, last recorded step: with periodic walls
                                 the step changes the momentum by exactly this     */
    double sor_residual;      /* Poisson residual after the last sweep of the last
                                 step that took it (recorded steps, and every step
                                 with sor_tol > 0)                                 */
    double sor_scale;         /* max|rhs| of that solve                             */
    int32_t sor_sweeps;       /* sweeps that solve ran                              */
    int32_t pad_;
    int64_t n_sor_noconv;     /* solves that ended above sor_tol, all steps        */
    double inlet_ubar;        /* mean velocity inside the nozzle measured by the
                                 adaptive inlet in the last step (0 without it)    */
} elbm_diag;

/* ABI version of the loaded library (ELBM_ABI_VERSION). */
uint32_t elbm_abi_version(void);

/* Validates params and boxes (copied), lays out the arena.  *out owns host
 * memory only; release it with elbm_destroy.  The model constants are those
 * of Sec. II (Shan-Chen couplings of Eq. sc, the Carreau law of Eq. carreau,
 * the charge models of Eqs. surface-q2 / surface-q3).  EINVAL on a bad value
 * (nothing is kept). */
elbm_status elbm_create(const elbm_params *params, const elbm_box *boxes, int32_t nboxes,
                        elbm_ctx **out);

/* Bytes of device memory the context needs in its arena (all fields of every
 * box, structure of arrays; see the layout notes in the library source). */
elbm_status elbm_required_bytes(const elbm_ctx *ctx, size_t *bytes);

/* Binds the caller-owned device arena (256-byte aligned, >= required bytes)
 * and a hipStream_t (NULL = the null stream).  Uploads the box tables and
 * clears the counters.  Synchronous. */
elbm_status elbm_bind(elbm_ctx *ctx, void *dev_arena, size_t bytes, void *hip_stream);

/* Sets the geometry and initial state of one box (synchronous):
 *  node_type [N] bytes; rho [C][N] initial component densities; u [3][N]
 *  initial velocity; phi [N] initial potential (Dirichlet nodes keep it);
 *  u_bc [3][N] inlet velocity (read at inlet nodes only; may be NULL);
 *  xi [C][19][N] jitter draws (may be NULL = no jitter); jitter amplitude.
 * node_type bytes are ELBM_NODE_* (NOZZLE only on fluid nodes; EINVAL otherwise).
 * Fluid nodes start at f = f_eq(rho, u) (1 + jitter * xi), inlet nodes at
 * f_eq(rho_in, u_bc) (at rest with an adaptive inlet), outlet nodes at
 * f_eq(rho_out, 0), solid nodes at 0.  Every step resets the inlet nodes as
 * elbm_params.inlet_mode says (the jet set-up of Sec. III.B); outlet nodes
 * keep theirs. */
elbm_status elbm_set_box(elbm_ctx *ctx, int32_t box, const uint8_t *node_type, const double *rho,
                         const double *u, const double *phi, const double *u_bc, const double *xi,
                         double jitter);

/* Enqueues nsteps time steps of every box on the bound stream (asynchronous):
 * each step is the update of Sec. II.C in the order of its summary (stream,
 * moments, charge of Eq. surface-q2/q3, Poisson solve of the Gauss law,
 * electric force Eq. force_el2, Shan-Chen force Eq. sc, alpha of Eq.
 * entropic, Carreau viscosity and beta of Eqs. strain2/carreau/beta,
 * collision Eq. lattice-b with the source of Eq. add).
 * record != 0: the last step also stores the recorded fields (component
 * densities, half-step velocity of Sec. II, alpha and its updates, the
 * electric-force sum and the Poisson residual) that the elbm_read_* and
 * elbm_diagnostics calls return.  Device conditions set the sticky word that
 * elbm_sync reports; EINVAL for nsteps < 0, ESTATE before bind. */
elbm_status elbm_step(elbm_ctx *ctx, int32_t nsteps, int32_t record);

/* enable != 0 (the default): elbm_step replays pairs of unrecorded steps as a
 * captured two-step hipGraph on the bound stream (built on first use, kept
 * with the context; never on the null stream or while timing).  enable == 0:
 * every kernel is launched directly.  Results are bitwise identical. */
elbm_status elbm_set_graphs(elbm_ctx *ctx, int32_t enable);

/* Waits for the stream and reports the sticky device error word since bind:
 * ELBM_ENONFINITE (a non-finite post-collision population), else
 * ELBM_ENEGPOP (a negative one, with ELBM_STRICT_NEGPOP), else ELBM_ENOCONV
 * (a Poisson solve above sor_tol, or with ELBM_STRICT_ALPHA an alpha
 * fallback: no root of Eq. entropic in the positivity interval or no
 * convergence).  elbm_last_error names the condition. */
elbm_status elbm_sync(elbm_ctx *ctx);

/* Reads (synchronising first) from the last recorded step:
 *  rho [C][N] component densities after streaming (zeroth moment of Eq.
 *  lattice-b's populations), u [3][N] half-step velocity
 *  sum_s (j_s + F_s/2) / sum_s rho_s (Sec. II, after Eq. add). */
elbm_status elbm_read_moments(elbm_ctx *ctx, int32_t box, double *rho, double *u);
/* potential phi [N] after the last step's Poisson solve (Sec. II, Gauss
 * law div(eps E) = q, E = E_ext - grad phi; Dirichlet nodes hold theirs) */
elbm_status elbm_read_potential(elbm_ctx *ctx, int32_t box, double *phi);
/* free charge q [N] of the last step, Eq. surface-q2 or surface-q3 (without
 * the neutralising background) */
elbm_status elbm_read_charge(elbm_ctx *ctx, int32_t box, double *q);
/* alpha [C][N] of Eq. entropic and its updates iters [C][N] (-1 = fallback)
 * of the last recorded step; zeros at non-fluid nodes.  iters may be NULL. */
elbm_status elbm_read_alpha(elbm_ctx *ctx, int32_t box, double *alpha, int32_t *iters);
/* current post-collision populations [C][19][N] of Eq. lattice-b (get) /
 * replace them (set): with elbm_set_potential, a checkpoint of the state */
elbm_status elbm_get_populations(elbm_ctx *ctx, int32_t box, double *f);
elbm_status elbm_set_populations(elbm_ctx *ctx, int32_t box, const double *f);
/* replaces the potential [N] (warm start of the next Poisson solve) */
elbm_status elbm_set_potential(elbm_ctx *ctx, int32_t box, const double *phi);

/* Conservation and solver diagnostics of one box (elbm_diag above): mass and
 * momentum of the current populations, alpha statistics and the electric-force
 * sum of the last recorded step, counters since bind.  Synchronous. */
elbm_status elbm_diagnostics(elbm_ctx *ctx, int32_t box, elbm_diag *out);

/* Phases of one step for elbm_timing. */
enum {
    ELBM_PHASE_DENSITY = 0,   /* pull + component densities                       */
    ELBM_PHASE_CHARGE = 1,    /* gradient, curvature, charge reductions, Poisson rhs */
    ELBM_PHASE_POISSON = 2,   /* red-black SOR sweeps (+ zero-mean gauge)          */
    ELBM_PHASE_EFIELD = 3,    /* |E|^2                                             */
    ELBM_PHASE_ALPHA = 4,     /* pull, entropic alpha, rheology (k_alpha)          */
    ELBM_PHASE_COLLIDE = 5,   /* forces, collision update, inlet nodes (k_collide) */
    ELBM_NPHASES = 6
};

/* Device timing of every phase: enable != 0 records HIP events on the bound
 * stream around each phase of each following step (a small overhead between
 * launches); enable == 0 stops and discards.  Host-side events only, no device
 * memory.  Without timing the alpha phase runs on a second stream of the
 * library, beside the charge, Poisson and E-field phases; with timing every
 * phase runs in order on the bound stream. */
elbm_status elbm_set_timing(elbm_ctx *ctx, int32_t enable);

/* Waits for the stream and returns the accumulated device milliseconds per
 * phase ms[ELBM_NPHASES] and the number of timed steps since timing was
 * enabled (either pointer may be NULL), then restarts the accumulation. */
elbm_status elbm_timing(elbm_ctx *ctx, double *ms, int64_t *steps);

/* ---- Learned starter of the alpha Newton iteration (ELBM_GUESS_MLP) ----
 * A 20 -> 32 -> 32 -> 1 SiLU network, BF16 weights and activations with FP32
 * accumulation on the matrix cores.  Input per node and component: the 19
 * ratios r_p = f_p/f_eq_p as z_p = (r_p - 1)/s and s = max_p |r_p - 1| (no
 * starter when a population or equilibrium entry is not positive or s is 0
 * or above 1); output y; starter alpha0 = 2 + s y.  In the update it serves
 * the nodes where the series starter is rejected (large non-equilibrium, at
 * interfaces); Newton then polishes to the same rule as every other starter.
 * Parameters: FP32 vector of 1761 floats, in order W1[32][20], b1[32],
 * W2[32][32], b2[32], w3[32], b3. */

/* Sets the parameters (host, n = 1761) and clears the optimiser state.  The
 * network approximates the root of Eqs. entropic / H that Newton polishes. */
elbm_status elbm_mlp_set_weights(elbm_ctx *ctx, const float *w, int64_t n);
/* Copies the current parameters to the host (n = 1761). */
elbm_status elbm_mlp_get_weights(elbm_ctx *ctx, float *w, int64_t n);
/* Inference on the bound stream: device X float [M][20] -> device Y float [M]. */
elbm_status elbm_mlp_forward(elbm_ctx *ctx, const void *dX, void *dY, int64_t M);
/* Gradient of L = (1/2M) sum_i (y_i - T_i)^2 over device X [M][20], T [M]
 * (synchronous): grad [1761] in parameter order and the loss, host pointers
 * (either may be NULL). */
elbm_status elbm_mlp_grad(elbm_ctx *ctx, const void *dX, const void *dT, int64_t M, float *grad,
                          float *loss);
/* For callers that cannot allocate (code under HIP graph capture, tight
 * training loops, harnesses that forbid hipMalloc): the gradient of
 * elbm_mlp_grad, enqueued on the bound stream without synchronising and
 * written to device memory dGrad, float [1762] (the 1761 gradient entries in
 * parameter order, then the loss).  Bitwise equal to elbm_mlp_grad's result.
 * It allocates nothing: its scratch (64 block partials of 2146 floats, 549 KB,
 * whatever M is) is a fixed device array of the library, one per GPU, kept
 * until the process ends and fully rewritten by every call; calls that
 * overlap on one GPU race for it.  EINVAL for NULL pointers or M <= 0. */
elbm_status elbm_mlp_grad_noalloc(elbm_ctx *ctx, const void *dX, const void *dT, int64_t M, void *dGrad);
/* steps (<= 4096) Adam steps (beta 0.9, 0.999, eps 1e-8, learning rate lr) on
 * consecutive batches of `batch` samples of device X [M][20], T [M], wrapping at
 * M (the caller shuffles); losses [steps] (host, may be NULL) receives each
 * batch loss.  Synchronous. */
elbm_status elbm_mlp_train(elbm_ctx *ctx, const void *dX, const void *dT, int64_t M, int32_t batch,
                           int32_t steps, float lr, float *losses);
/* Training samples from the current state of one box (the populations the
 * next step pulls): for node n and component s at index s * N + n, the
 * starter input feat [.][20] (z, s), the target (alpha* - 2)/s with alpha*
 * the plain Newton root from 2, the scale s, and a flag: 0 at non-fluid
 * nodes, without features, or where the plain solve fell back; 1 a usable
 * sample; 2 a usable sample at a node the learned starter serves (the series
 * starter is rejected there).
 * Device pointers: float [C*N][20], float [C*N], float [C*N], int32 [C*N].
 * Synchronous. */
elbm_status elbm_alpha_samples(elbm_ctx *ctx, int32_t box, void *dFeat, void *dTarget, void *dScale,
                               void *dValid);

/* ---- Launch mapping and its autotuner ----
 * xcd_remap: 1 orders the node blocks so that each of the 8 XCDs runs one
 * contiguous range of tiles (neighbouring tiles share an L2); 0 keeps the
 * hardware's round-robin order.  graph_steps: steps captured in one HIP graph
 * (even, 2..64).  tile: the block tile of the alpha kernel (the first half
 * of the collision), 0 = 256 consecutive nodes
 * (a 64-thread wave is a run along x), 1 = 8x8x4 nodes (waves 8x8x1),
 * 2 = 8x4x8 (waves 8x4x2), 3 = 4x4x16 (waves 4x4x4): 3-D waves gather the
 * nodes whose alpha needs many Newton updates (at interfaces) into fewer
 * waves.  sweep_priority: 1 raises the instruction-issue priority of the
 * waves of the field chain after the densities (gradient, interface, charge,
 * SOR sweeps, gauge, E field), which runs on the bound stream while the alpha
 * kernel runs on the library's second stream: it helps when that chain is
 * the longer of the two branches, 0 (hardware default) when alpha is.
 * stencil_lds: 1 stages the neighbour values of the density-gradient and
 * E-field stencils in LDS (each 256-node block loads, for the z offsets -1, 0,
 * +1 of the stencil, its own index range widened by nx + 1 nodes on either
 * side, then reads those slabs in place of per-direction loads); it needs the
 * slabs of the widest box, (D3Q19: 3, D2Q9: 1) x (256 + 2 (nx + 1)) field
 * values, within 32 KB, else ELBM_EINVAL.  0 (default) reads each neighbour
 * from memory.  None changes any result: per-node arithmetic and the order
 * of every reduction are the same under all mappings. */
typedef struct elbm_launch {
  int32_t xcd_remap;
  int32_t graph_steps;
  int32_t tile;
  int32_t sweep_priority;
  int32_t stencil_lds;
} elbm_launch;
#define ELBM_TUNE_CANDIDATES 11
/* Sets / reads the launch mapping (synchronises the bound stream; drops the
 * captured graphs). */
elbm_status elbm_set_launch(elbm_ctx *ctx, const elbm_launch *launch);
elbm_status elbm_get_launch(const elbm_ctx *ctx, elbm_launch *launch);
/* Chooses the mapping in four passes, each timing its candidates over
 * steps_per_trial steps (rounded up to a multiple of 16) with HIP events on
 * the bound stream, in two rounds (forward, then reverse order; a
 * candidate's time is the mean of its two rounds), and keeping the fastest for the
 * next pass: tile 0..3 (with xcd_remap 0, graph_steps 2, sweep_priority
 * 0), then xcd_remap 0, 1, then sweep_priority 0, 1, then graph_steps 2, 4,
 * 8.  best (may be NULL) receives the result;
 * ms_per_step [ELBM_TUNE_CANDIDATES] (may be NULL) each candidate's ms per
 * step in that order.  The trial steps are ordinary steps: the state
 * advances by 22 trial + 60 steps (each of the 22 trials first runs one
 * graph's worth of steps to capture it).
 * Synchronous; phase timing must be off. */
elbm_status elbm_autotune(elbm_ctx *ctx, int32_t steps_per_trial, elbm_launch *best, double *ms_per_step);

/* Message of the last failing call on this context (never NULL). */
const char *elbm_last_error(const elbm_ctx *ctx);

/* Releases the host state; the arena stays the caller's. */
void elbm_destroy(elbm_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* ELBM_H */
