/*
 * Plain FP64 CPU oracle of the per-time-step lattice update of the entropic
 * lattice Boltzmann model for charged leaky-dielectric multiphase fluids
 * (Lauricella, Melchionna, Montessori, Pisignano, Pontrelli, Succi,
 * "Entropic Lattice Boltzmann Model for Charged Leaky Dielectric Multiphase
 * Fluids in Electrified Jets", arXiv:1612.05404).
 *
 * TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
 * CPU-baseline leg call it; the product path never does.  It shares no code,
 * header, table or helper with the HIP library: both are written from the
 * paper independently.
 *
 * Scalar loops, OpenMP over z only, compensated (Neumaier) sums for every
 * global reduction, no blocking, no fusion.  The paper's model is 2-D D2Q9
 * and single-component; this oracle runs the 3-D D3Q19 lattice with one or
 * two Shan-Chen components, so the single-component model is the ncomp = 1
 * special case.
 *
 * Step order (Sec. II.C, "Summary of the model"): the five stages depend
 * only on the post-streaming populations of the current step, so they are
 * evaluated here as stream -> moments -> fields -> charge (Eq. surface-q2 /
 * surface-q3) -> Poisson -> electric field and force (Eq. force_el2) ->
 * Shan-Chen force (Eq. sc) -> alpha (Eq. entropic) -> Carreau rheology
 * (Eqs. strain2, carreau, beta) -> collision with the exact-difference
 * source (Eqs. lattice-b, add).
 *
 * Parity unpinned: none of the functions below is left without a pin in the
 * CPU test-suite; see the tests for each pin.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define QMAX 19
#define CS2 (1.0 / 3.0)

/* Lattices (Sec. II, Eq. lattice-b and the weights below it).  D3Q19:
 * rest, the 6 face neighbours, the 12 edge neighbours; the paper's D2Q9
 * weights 4/9, 1/9, 1/36 become 1/3, 1/18, 1/36 in 3-D (same c_s^2 = 1/3).
 * D2Q9 (the paper's own lattice): rest, 4 axis and 4 diagonal neighbours in
 * the x-y plane (c_z = 0; a 2-D box has nz = 1, bounded in z).  Opposite
 * directions sit at adjacent (odd, even) indices in both. */
typedef struct {
    int q;
    int c[QMAX][3];
    double w[QMAX];
} ora_lat;

static const ora_lat LAT_D3Q19 = {
    19,
    {{0, 0, 0},
     {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
     {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
     {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
     {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}},
    {1.0 / 3.0,
     1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
     1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
     1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0}};

static const ora_lat LAT_D2Q9 = {
    9,
    {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
     {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}},
    {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
     1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0}};

static const ora_lat *lattice_of(int id) { return id == 1 ? &LAT_D2Q9 : &LAT_D3Q19; }

/* The state's lattice under the names the stage functions use. */
#define LAT_LOCALS(st)                                                                   \
    const int Q = (st)->Q;                                                               \
    const int(*CV)[3] = (st)->lat->c;                                                    \
    const double *WV = (st)->lat->w;                                                     \
    (void)Q;                                                                             \
    (void)CV;                                                                            \
    (void)WV

static int opposite(int p) { return p == 0 ? 0 : ((p & 1) ? p + 1 : p - 1); }

enum { T_FLUID = 0, T_SOLID = 1, T_INLET = 2, T_OUTLET = 3, T_DIRICHLET = 4, T_NOZZLE = 8 };

typedef struct {
    int32_t nx, ny, nz, ncomp;
    int32_t periodic[3];
    int32_t carreau, curvature, electrostriction, charge_model;
    int32_t sor_sweeps, newton_max, nthreads, pad_;
    double G[2][2];
    double Gw[2][2];
    double nu0, nu_inf, lam, n_flow;
    double Q_b, Q_s, xi_b, xi_s, K_d, rho_th, w_theta;
    double E_ext[3];
    double sor_omega, newton_rtol;
    double rho_in[2], rho_out[2];
    /* Poisson stop rule: sor_tol > 0 ends the sweeps once the residual is at
     * most sor_tol * max|rhs| (checked after every sor_check_every sweeps when
     * that is > 0, and after the last one); sor_tol = 0: exactly sor_sweeps */
    double sor_tol;
    int32_t sor_check_every;
    int32_t lattice;  /* 0: D3Q19, 1: D2Q9 (nz = 1, bounded in z) */
    /* inlet: 0 the neighbour-density velocity inlet (u_bc as given); 1 + a:
     * the paper's jet inlet, density rho_in and velocity ubar * u_bc, ubar the
     * mean velocity along axis a inside the nozzle (fluid nodes marked
     * T_NOZZLE), measured every step */
    int32_t inlet_mode;
    int32_t pad2_;
} ora_params;

typedef struct {
    ora_params P;
    const ora_lat *lat;
    int Q;
    int64_t N;
    int C;
    uint8_t *type;
    double *f;      /* post-collision populations (state)  [C][Q][N] */
    double *fn;     /* next post-collision populations      [C][Q][N] */
    double *fp;     /* post-streaming (pulled) populations  [C][Q][N] */
    double *rho;    /* [C][N] */
    double *jm;     /* [C][3][N] */
    double *psi;    /* [C][N] */
    double *grad;   /* [3][N]  gradient of the liquid density */
    double *nhat;   /* [3][N] */
    double *K;      /* [N] mean curvature */
    double *bulk;   /* [N] rho_A theta */
    double *surf;   /* [N] |grad rho_A|^2 (1 + (K/K_d)^(1/4)) */
    double *q;      /* [N] free charge */
    double *phi;    /* [N] */
    double *rhs;    /* [N] */
    double *E;      /* [3][N] */
    double *E2;     /* [N] */
    double *Fel;    /* [3][N] total electric force */
    double *F;      /* [C][3][N] total force per component */
    double *alpha;  /* [C][N] */
    int32_t *iters; /* [C][N] */
    double *nu;     /* [C][N] viscosity used in the collision */
    double *uph;    /* [3][N] half-step barycentric velocity */
    double *u_bc;   /* [3][N] inlet velocity */
    double qbar;
    double ubar;    /* mean velocity inside the nozzle of this step's moments */
    double Sb, Ss;
    int64_t nfallback;
    int64_t nerr_nonfinite, nerr_negative;
    int has_dirichlet;
    int64_t n_unknown;
    /* Poisson solve of the last step: residual max|sum_f eps_f (phi_nb - phi)
     * - rhs| over the unknown nodes after the last sweep, its scale max|rhs|,
     * sweeps done; steps whose solve missed the tolerance */
    double sor_res, sor_scale;
    int32_t sor_done;
    int64_t sor_noconv;
} ora_state;

/* ---------------------------------------------------------------- sums */
typedef struct { double s, c; } nsum;
static void ns_add(nsum *a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}
static double ns_val(const nsum *a) { return a->s + a->c; }

/* ------------------------------------------------------------ geometry */
static int64_t node_index(const ora_state *s, int x, int y, int z) {
    return (int64_t)x + (int64_t)s->P.nx * ((int64_t)y + (int64_t)s->P.ny * z);
}

/* Neighbour r + d, wrapping periodic axes; -1 when it leaves the domain. */
static int64_t neighbour(const ora_state *s, int x, int y, int z, int dx, int dy, int dz) {
    int n[3] = {s->P.nx, s->P.ny, s->P.nz};
    int c[3] = {x + dx, y + dy, z + dz};
    for (int a = 0; a < 3; ++a) {
        if (c[a] < 0 || c[a] >= n[a]) {
            if (!s->P.periodic[a]) return -1;
            c[a] = (c[a] + n[a]) % n[a];
        }
    }
    return node_index(s, c[0], c[1], c[2]);
}

static int kind(const ora_state *s, int64_t n) { return s->type[n] & 3; }
static int is_solid(const ora_state *s, int64_t n) { return n < 0 || kind(s, n) == T_SOLID; }

/* ---------------------------------------------------- node-level maths */

/* Second-order equilibrium (Sec. II, the Mach expansion below Eq. lattice-b). */
static void feq_lat(const ora_lat *L, double rho, const double u[3], double *out) {
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int p = 0; p < L->q; ++p) {
        double cu = L->c[p][0] * u[0] + L->c[p][1] * u[1] + L->c[p][2] * u[2];
        out[p] = L->w[p] * rho * (1.0 + cu / CS2 + (cu * cu - CS2 * uu) / (2.0 * CS2 * CS2));
    }
}
void ora_feq(double rho, const double u[3], double out[19]) { feq_lat(&LAT_D3Q19, rho, u, out); }
void ora_feq_lat(int lattice, double rho, const double u[3], double *out) {
    feq_lat(lattice_of(lattice), rho, u, out);
}

/* phi(y) = (1+y) ln(1+y) - y, accurate for small |y| (its Taylor series
 * sum_{k>=2} (-1)^k y^k / (k(k-1)) summed to convergence). */
static double phi_fn(double y) {
    if (fabs(y) < 0.25) {
        double term = y * y, sum = 0.0;
        for (int k = 2; k < 200; ++k) {
            double t = term / ((double)k * (double)(k - 1));
            if (k & 1) t = -t;
            double ns = sum + t;
            if (ns == sum) break;
            sum = ns;
            term *= y;
        }
        return sum;
    }
    return (1.0 + y) * log1p(y) - y;
}

/*
 * Entropic over-relaxation (Eqs. entropic, H): alpha is the non-trivial
 * root of H(f + alpha (f_eq - f)) = H(f), H(f) = sum_p f_p ln(f_p / w_p).
 * With Delta = f_eq - f and x_p = Delta_p / f_p the difference is, exactly,
 *   g(alpha) = sum_p f_p phi(alpha x_p) + alpha L,
 *   L = sum_p Delta_p ln(f_p / (w_p rho)),
 * using sum_p Delta_p = 0 (f and f_eq carry the same density).  A
 * non-positive population leaves H(f) undefined: fallback.
 * g is convex on the positivity interval 0 < alpha < alpha_max, g(0) = 0,
 * g'(0) = L.  At the upper end the population that vanishes contributes
 * f_p phi(-1) = f_p (finite), so g(alpha_max-) is finite: a root exists iff
 * L < 0 and g(alpha_max-) > 0, and it is then unique.
 * Newton from alpha0 (2 = the BGK limit, or a supplied guess); a step that
 * leaves the positivity interval is halved toward its edge, and the first
 * time one leaves it at the top, g(alpha_max-) is evaluated: not positive
 * means no root.  Convergence when |g| <= rtol * sum_p f_p phi(alpha x_p) or
 * the step stalls at rounding.
 * No root or no convergence: alpha = min(2, 0.99 alpha_max), flagged.
 * Returns the number of Newton updates (>= 0) or -1 on fallback.
 */
/* g at the top of the positivity interval (see ora_alpha): phi(-1) = 1. */
static double g_at_alpha_max(int Q, const double *f, const double *x, double L, double amax) {
    double S = 0.0;
    for (int p = 0; p < Q; ++p) {
        double y = amax * x[p];
        S += f[p] * (y > -1.0 ? phi_fn(y) : 1.0);
    }
    return S + amax * L;
}

static double alpha_lat(const ora_lat *lat, const double *f, const double *feq, double rho,
                        double alpha0, double rtol, int maxit, int *iters_out) {
    const int Q = lat->q;
    const double *WV = lat->w;
    double D[QMAX], x[QMAX];
    double xmax = 0.0, amax = INFINITY;
    int nonpos = 0;
    for (int p = 0; p < Q; ++p) {
        D[p] = feq[p] - f[p];
        x[p] = D[p] / f[p];
        if (!(f[p] > 0.0)) nonpos = 1;
        if (fabs(x[p]) > xmax) xmax = fabs(x[p]);
        if (x[p] < 0.0 && -1.0 / x[p] < amax) amax = -1.0 / x[p];
    }
    if (nonpos) {  /* H(f) is undefined for a non-positive population */
        *iters_out = -1;
        return fmin(2.0, 0.99 * amax);
    }
    if (xmax < 1e-12) { *iters_out = 0; return 2.0; }
    /* L = sum_p Delta_p ln(f_p / (w_p rho)): defined for every f > 0, also
     * where the polynomial equilibrium is negative */
    double L = 0.0;
    for (int p = 0; p < Q; ++p) L += D[p] * log1p((f[p] - WV[p] * rho) / (WV[p] * rho));
    double a = alpha0;
    if (!(a > 0.0 && a < amax)) a = 0.5 * (amax < 4.0 ? amax : 4.0);
    if (L < 0.0) {
        int probed = 0;
        for (int it = 0; it <= maxit; ++it) {
            double S = 0.0, gp = L;
            for (int p = 0; p < Q; ++p) {
                S += f[p] * phi_fn(a * x[p]);
                gp += D[p] * log1p(a * x[p]);
            }
            double g = S + a * L;
            if (fabs(g) <= rtol * S) { *iters_out = it; return a; }
            if (it == maxit) break;
            double an;
            if (gp > 0.0) an = a - g / gp;
            else an = 2.0 * a;                      /* left of the minimum of g */
            if (an >= amax) {
                if (!probed) {  /* leaving at the top: is there a root at all? */
                    probed = 1;
                    if (!(g_at_alpha_max(Q, f, x, L, amax) > 0.0)) break;
                }
                an = 0.5 * (a + amax);
            }
            if (an <= 0.0) an = 0.5 * a;
            if (fabs(an - a) <= 4.0 * DBL_EPSILON * a) { *iters_out = it + 1; return an; }
            a = an;
        }
    }
    *iters_out = -1;
    return fmin(2.0, 0.99 * amax);
}

double ora_alpha(const double f[19], const double feq[19], const double u[3], double rho,
                 double alpha0, double rtol, int maxit, int *iters_out) {
    (void)u;
    return alpha_lat(&LAT_D3Q19, f, feq, rho, alpha0, rtol, maxit, iters_out);
}
double ora_alpha_lat(int lattice, const double *f, const double *feq, double rho, double alpha0,
                     double rtol, int maxit, int *iters_out) {
    return alpha_lat(lattice_of(lattice), f, feq, rho, alpha0, rtol, maxit, iters_out);
}

/* Largest |eigenvalue| of a symmetric 3x3 matrix (the matrix 2-norm) by
 * cyclic Jacobi rotations; m = {xx, yy, zz, xy, xz, yz}. */
double ora_sym3_norm2(const double m6[6]) {
    double a[3][3] = {{m6[0], m6[3], m6[4]}, {m6[3], m6[1], m6[5]}, {m6[4], m6[5], m6[2]}};
    for (int sweep = 0; sweep < 50; ++sweep) {
        double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
        double diag = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
        if (off <= 1e-40 * diag || off == 0.0) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (a[p][q] == 0.0) continue;
                double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < 3; ++k) { /* A <- A J */
                    double akp = a[k][p], akq = a[k][q];
                    a[k][p] = c * akp - sn * akq;
                    a[k][q] = sn * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) { /* A <- J^T A */
                    double apk = a[p][k], aqk = a[q][k];
                    a[p][k] = c * apk - sn * aqk;
                    a[q][k] = sn * apk + c * aqk;
                }
            }
    }
    double r = fabs(a[0][0]);
    if (fabs(a[1][1]) > r) r = fabs(a[1][1]);
    if (fabs(a[2][2]) > r) r = fabs(a[2][2]);
    return r;
}

/* Carreau law (Eq. carreau). */
double ora_carreau_nu(double gd, double nu0, double nu_inf, double lam, double n) {
    return nu_inf + (nu0 - nu_inf) * pow(1.0 + (lam * gd) * (lam * gd), 0.5 * (n - 1.0));
}

/*
 * Shear rate (Eq. strain2): gamma = Pi / (rho tau(gamma) c_s^2) with
 * tau = 1/(alpha beta(nu(gamma))), beta = c_s^2/(2 nu + c_s^2) (Eq. beta), i.e.
 * h(gamma) = rho (2 nu(gamma) + c_s^2) gamma - alpha Pi = 0.  h is strictly
 * increasing for n > 0, h(0) <= 0 and h(hi) >= 0 with
 * hi = alpha Pi / (rho (2 nu_inf + c_s^2)); Newton kept inside the bracket,
 * bisection when it leaves it.  Pi = 0 or rho <= 0: gamma = 0 (nu = nu0).
 */
double ora_shear_rate(double Pn, double rho, double alpha, double nu0, double nu_inf,
                      double lam, double n) {
    /* no positive root without stress, or at a non-positive density (only
     * reachable after negative populations): the shear rate is taken as 0 */
    if (!(Pn > 0.0) || !(rho > 0.0)) return 0.0;
    double lo = 0.0, hi = alpha * Pn / (rho * (2.0 * nu_inf + CS2));
    double g = 0.5 * hi;
    for (int it = 0; it < 200; ++it) {
        double s = 1.0 + (lam * g) * (lam * g);
        double nu = nu_inf + (nu0 - nu_inf) * pow(s, 0.5 * (n - 1.0));
        double h = rho * (2.0 * nu + CS2) * g - alpha * Pn;
        if (h > 0.0) hi = g; else lo = g;
        double dh = rho * (2.0 * nu_inf + CS2 + 2.0 * (nu0 - nu_inf) * pow(s, 0.5 * (n - 3.0)) *
                                                    (1.0 + n * (lam * g) * (lam * g)));
        double gn = g - h / dh;
        if (!(gn > lo && gn < hi)) gn = 0.5 * (lo + hi);
        if (fabs(gn - g) <= 1e-15 * g || hi - lo <= 1e-16 * hi) return gn;
        g = gn;
    }
    return g;
}

/* ------------------------------------------------------------- the box */
static void *xcalloc(size_t n, size_t sz) { return calloc(n ? n : 1, sz); }

ora_state *ora_create(const ora_params *P, const uint8_t *type, const double *phi0,
                      const double *u_bc) {
    ora_state *s = (ora_state *)calloc(1, sizeof(ora_state));
    s->lat = lattice_of(P->lattice);
    s->Q = s->lat->q;
    LAT_LOCALS(s);
    s->P = *P;
    s->C = P->ncomp;
    s->N = (int64_t)P->nx * P->ny * P->nz;
    int64_t N = s->N, C = s->C;
    s->type = (uint8_t *)xcalloc(N, 1);
    memcpy(s->type, type, N);
    s->f = xcalloc(C * Q * N, sizeof(double));
    s->fn = xcalloc(C * Q * N, sizeof(double));
    s->fp = xcalloc(C * Q * N, sizeof(double));
    s->rho = xcalloc(C * N, sizeof(double));
    s->jm = xcalloc(C * 3 * N, sizeof(double));
    s->psi = xcalloc(C * N, sizeof(double));
    s->grad = xcalloc(3 * N, sizeof(double));
    s->nhat = xcalloc(3 * N, sizeof(double));
    s->K = xcalloc(N, sizeof(double));
    s->bulk = xcalloc(N, sizeof(double));
    s->surf = xcalloc(N, sizeof(double));
    s->q = xcalloc(N, sizeof(double));
    s->phi = xcalloc(N, sizeof(double));
    s->rhs = xcalloc(N, sizeof(double));
    s->E = xcalloc(3 * N, sizeof(double));
    s->E2 = xcalloc(N, sizeof(double));
    s->Fel = xcalloc(3 * N, sizeof(double));
    s->F = xcalloc(C * 3 * N, sizeof(double));
    s->alpha = xcalloc(C * N, sizeof(double));
    s->iters = xcalloc(C * N, sizeof(int32_t));
    s->nu = xcalloc(C * N, sizeof(double));
    s->uph = xcalloc(3 * N, sizeof(double));
    s->u_bc = xcalloc(3 * N, sizeof(double));
    if (phi0) memcpy(s->phi, phi0, N * sizeof(double));
    if (u_bc) memcpy(s->u_bc, u_bc, 3 * N * sizeof(double));
    s->has_dirichlet = 0;
    s->n_unknown = 0;
    for (int64_t n = 0; n < N; ++n) {
        if (type[n] & T_DIRICHLET) s->has_dirichlet = 1;
        else s->n_unknown++;
    }
#ifdef _OPENMP
    if (P->nthreads > 0) omp_set_num_threads(P->nthreads);
#endif
    return s;
}

void ora_destroy(ora_state *s) {
    if (!s) return;
    void *ptrs[] = {s->type, s->f, s->fn, s->fp, s->rho, s->jm, s->psi, s->grad, s->nhat,
                    s->K, s->bulk, s->surf, s->q, s->phi, s->rhs, s->E, s->E2, s->Fel, s->F,
                    s->alpha, s->iters, s->nu, s->uph, s->u_bc};
    for (size_t i = 0; i < sizeof(ptrs) / sizeof(ptrs[0]); ++i) free(ptrs[i]);
    free(s);
}

/* Initial boundary-node populations: inlet nodes f_eq(rho_in, u_bc), outlet
 * nodes f_eq(rho_out, 0).  Neither streams nor collides; outlet nodes keep
 * theirs, inlet nodes are reset every step (see inlet_populations). */
static void boundary_populations(ora_state *s, int64_t n, int sigma, double *out) {
    LAT_LOCALS(s);
    double u[3] = {0, 0, 0};
    double r;
    if (kind(s, n) == T_INLET) {
        const double sc = s->P.inlet_mode > 0 ? 0.0 : 1.0;  /* the adaptive inlet starts from rest */
        u[0] = sc * s->u_bc[n]; u[1] = sc * s->u_bc[s->N + n]; u[2] = sc * s->u_bc[2 * s->N + n];
        r = s->P.rho_in[sigma];
    } else {
        r = s->P.rho_out[sigma];
    }
    feq_lat(s->lat, r, u, out);
}

/* Initial state: f = f_eq(rho, u) (1 + amp * xi) at fluid nodes;
 * boundary nodes get their fixed equilibria; solid nodes hold zeros. */
void ora_init(ora_state *s, const double *rho0, const double *u0, const double *xi, double amp) {
    LAT_LOCALS(s);
    int64_t N = s->N;
    for (int sg = 0; sg < s->C; ++sg)
        for (int64_t n = 0; n < N; ++n) {
            double fe[QMAX];
            int k = kind(s, n);
            if (k == T_SOLID) {
                for (int p = 0; p < Q; ++p) s->f[((int64_t)sg * Q + p) * N + n] = 0.0;
                continue;
            }
            if (k == T_INLET || k == T_OUTLET) {
                boundary_populations(s, n, sg, fe);
                for (int p = 0; p < Q; ++p) s->f[((int64_t)sg * Q + p) * N + n] = fe[p];
                continue;
            }
            double u[3] = {u0[n], u0[N + n], u0[2 * N + n]};
            feq_lat(s->lat, rho0[(int64_t)sg * N + n], u, fe);
            for (int p = 0; p < Q; ++p) {
                double j = xi ? xi[((int64_t)sg * Q + p) * N + n] : 0.0;
                s->f[((int64_t)sg * Q + p) * N + n] = fe[p] * (1.0 + amp * j);
            }
        }
    memcpy(s->fn, s->f, (size_t)s->C * Q * N * sizeof(double));
}

/* -------------------------------------------------------- step stages */

/* Streaming (left-hand side of Eq. lattice-b) by pulling, halfway
 * bounce-back at solid nodes; moments rho = sum f, j = sum c f. */
static void stream_and_moments(ora_state *s) {
    LAT_LOCALS(s);
    const int64_t N = s->N;
    const int C = s->C;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < s->P.nz; ++z)
        for (int y = 0; y < s->P.ny; ++y)
            for (int x = 0; x < s->P.nx; ++x) {
                int64_t n = node_index(s, x, y, z);
                int k = kind(s, n);
                for (int sg = 0; sg < C; ++sg) {
                    double *fp = s->fp + (int64_t)sg * Q * N;
                    const double *fs = s->f + (int64_t)sg * Q * N;
                    if (k == T_SOLID) {
                        for (int p = 0; p < Q; ++p) fp[p * N + n] = 0.0;
                    } else if (k == T_INLET || k == T_OUTLET) {
                        for (int p = 0; p < Q; ++p) fp[p * N + n] = fs[p * N + n];
                    } else {
                        for (int p = 0; p < Q; ++p) {
                            int64_t src = neighbour(s, x, y, z, -CV[p][0], -CV[p][1], -CV[p][2]);
                            if (is_solid(s, src)) fp[p * N + n] = fs[opposite(p) * N + n];
                            else fp[p * N + n] = fs[p * N + src];
                        }
                    }
                    double r = 0.0, j0 = 0.0, j1 = 0.0, j2 = 0.0;
                    for (int p = 0; p < Q; ++p) {
                        double v = fp[p * N + n];
                        r += v;
                        j0 += CV[p][0] * v;
                        j1 += CV[p][1] * v;
                        j2 += CV[p][2] * v;
                    }
                    s->rho[(int64_t)sg * N + n] = r;
                    s->jm[((int64_t)sg * 3 + 0) * N + n] = j0;
                    s->jm[((int64_t)sg * 3 + 1) * N + n] = j1;
                    s->jm[((int64_t)sg * 3 + 2) * N + n] = j2;
                    s->psi[(int64_t)sg * N + n] = (k == T_SOLID) ? 0.0 : -expm1(-r);
                }
            }
    /* the jet inlet's measurement (Sec. III.B): mean velocity of the fluid in
     * the nozzle, total momentum along the inlet axis over total mass */
    s->ubar = 0.0;
    if (s->P.inlet_mode > 0) {
        const int a = s->P.inlet_mode - 1;
        double jsum = 0.0, msum = 0.0;
        for (int64_t n = 0; n < N; ++n) {
            if (kind(s, n) != T_FLUID || !(s->type[n] & T_NOZZLE)) continue;
            for (int sg = 0; sg < C; ++sg) {
                jsum += s->jm[((int64_t)sg * 3 + a) * N + n];
                msum += s->rho[(int64_t)sg * N + n];
            }
        }
        s->ubar = msum > 0.0 ? jsum / msum : 0.0;
    }
}

/* Isotropic 19-point gradient (1/c_s^2) sum_p w_p c_p X(r + c_p).
 * mode 0: a solid or outside neighbour takes the centre value;
 * mode 1: only an outside neighbour takes the centre value. */
static void gradient19(const ora_state *s, const double *X, int x, int y, int z, int mode,
                       double out[3]) {
    LAT_LOCALS(s);
    int64_t n = node_index(s, x, y, z);
    double g0 = 0, g1 = 0, g2 = 0;
    for (int p = 1; p < Q; ++p) {
        int64_t m = neighbour(s, x, y, z, CV[p][0], CV[p][1], CV[p][2]);
        double v;
        if (m < 0 || (mode == 0 && kind(s, m) == T_SOLID)) v = X[n];
        else v = X[m];
        g0 += WV[p] * CV[p][0] * v;
        g1 += WV[p] * CV[p][1] * v;
        g2 += WV[p] * CV[p][2] * v;
    }
    out[0] = g0 / CS2; out[1] = g1 / CS2; out[2] = g2 / CS2;
}

/* Interface geometry for the charge model: gradient of the liquid density,
 * normal n = grad rho / |grad rho|, mean curvature (Eq. surface-curvature,
 * with the sign that makes a convex drop positive: K = -div n), the smoothed
 * Heaviside theta and the two charge weights. */
static void interface_fields(ora_state *s) {
    LAT_LOCALS(s);
    const int64_t N = s->N;
    const double *rA = s->rho;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < s->P.nz; ++z)
        for (int y = 0; y < s->P.ny; ++y)
            for (int x = 0; x < s->P.nx; ++x) {
                int64_t n = node_index(s, x, y, z);
                double g[3] = {0, 0, 0};
                if (kind(s, n) != T_SOLID) gradient19(s, rA, x, y, z, 0, g);
                s->grad[n] = g[0]; s->grad[N + n] = g[1]; s->grad[2 * N + n] = g[2];
                double m = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
                for (int a = 0; a < 3; ++a) s->nhat[a * N + n] = (m > 1e-12) ? g[a] / m : 0.0;
            }
#pragma omp parallel for schedule(static)
    for (int z = 0; z < s->P.nz; ++z)
        for (int y = 0; y < s->P.ny; ++y)
            for (int x = 0; x < s->P.nx; ++x) {
                int64_t n = node_index(s, x, y, z);
                if (kind(s, n) == T_SOLID) {
                    s->K[n] = 0.0; s->bulk[n] = 0.0; s->surf[n] = 0.0;
                    continue;
                }
                double div = 0.0;
                for (int p = 1; p < Q; ++p) {
                    int64_t m = neighbour(s, x, y, z, CV[p][0], CV[p][1], CV[p][2]);
                    int64_t src = (m < 0 || kind(s, m) == T_SOLID) ? n : m;
                    div += WV[p] * (CV[p][0] * s->nhat[src] + CV[p][1] * s->nhat[N + src] +
                                    CV[p][2] * s->nhat[2 * N + src]);
                }
                double K = -div / CS2;
                s->K[n] = K;
                double theta = 0.5 * (1.0 + tanh((rA[n] - s->P.rho_th) / s->P.w_theta));
                s->bulk[n] = rA[n] * theta;
                double g2 = s->grad[n] * s->grad[n] + s->grad[N + n] * s->grad[N + n] +
                            s->grad[2 * N + n] * s->grad[2 * N + n];
                double wK = 1.0;
                if (s->P.curvature) wK += pow(fmax(K, 0.0) / s->P.K_d, 0.25);
                s->surf[n] = g2 * wK;
            }
}

/* Free charge: Eq. surface-q2 (conserving, normalised by the two global
 * integrals) or Eq. surface-q3 (generator-connected, fixed xi_b, xi_s). */
static void charge(ora_state *s) {
    const int64_t N = s->N;
    if (s->P.charge_model == 0) {
        nsum sb = {0, 0}, ss = {0, 0};
        for (int64_t n = 0; n < N; ++n) { ns_add(&sb, s->bulk[n]); ns_add(&ss, s->surf[n]); }
        s->Sb = ns_val(&sb); s->Ss = ns_val(&ss);
        for (int64_t n = 0; n < N; ++n) {
            double q = 0.0;
            if (s->Sb > 0.0) q += s->P.Q_b * s->bulk[n] / s->Sb;
            if (s->Ss > 0.0) q += s->P.Q_s * s->surf[n] / s->Ss;
            s->q[n] = q;
        }
    } else {
        for (int64_t n = 0; n < N; ++n) s->q[n] = s->P.xi_b * s->bulk[n] + s->P.xi_s * s->surf[n];
    }
}

static const int FACE[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};

/* Right-hand side of the discrete Gauss law (Sec. II: div(eps E) = q with
 * E = E_ext - grad phi, eps = 1 + rho_A), written per node as
 *   sum_f eps_f (phi_nb - phi) = sum_f eps_f E_ext . e_f - (q - qbar),
 * the sums over the six faces f that stay in the domain, eps_f the mean of
 * the two node permittivities, e_f the face's unit vector.  The first sum
 * is the outward flux of eps E_ext through the node's faces; qbar is the
 * uniform neutralising charge, the mean of q over the Poisson-unknown
 * nodes.  Returns qbar. */
double ora_poisson_rhs(const ora_state *s, const double *eps, const double *q, double *rhs) {
    nsum qs = {0, 0};
    for (int64_t n = 0; n < s->N; ++n)
        if (!(s->type[n] & T_DIRICHLET)) ns_add(&qs, q[n]);
    const double qbar = s->n_unknown ? ns_val(&qs) / (double)s->n_unknown : 0.0;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < s->P.nz; ++z)
        for (int y = 0; y < s->P.ny; ++y)
            for (int x = 0; x < s->P.nx; ++x) {
                int64_t n = node_index(s, x, y, z);
                double r = -(q[n] - qbar);
                for (int f = 0; f < 6; ++f) {
                    int64_t m = neighbour(s, x, y, z, FACE[f][0], FACE[f][1], FACE[f][2]);
                    if (m < 0) continue;
                    double ef = 0.5 * (eps[n] + eps[m]);
                    r += ef * (s->P.E_ext[0] * FACE[f][0] + s->P.E_ext[1] * FACE[f][1] +
                               s->P.E_ext[2] * FACE[f][2]);
                }
                rhs[n] = r;
            }
    return qbar;
}

/* Largest residual |sum_f eps_f (phi_nb - phi) - rhs| over the unknown
 * nodes; *scale (may be NULL) receives max|rhs| over the same nodes. */
double ora_poisson_residual(const ora_state *s, const double *eps, const double *rhs,
                            const double *phi, double *scale) {
    double rmax = 0.0, smax = 0.0;
    for (int z = 0; z < s->P.nz; ++z)
        for (int y = 0; y < s->P.ny; ++y)
            for (int x = 0; x < s->P.nx; ++x) {
                int64_t n = node_index(s, x, y, z);
                if (s->type[n] & T_DIRICHLET) continue;
                double acc = 0.0;
                for (int f = 0; f < 6; ++f) {
                    int64_t m = neighbour(s, x, y, z, FACE[f][0], FACE[f][1], FACE[f][2]);
                    if (m < 0) continue;
                    acc += 0.5 * (eps[n] + eps[m]) * (phi[m] - phi[n]);
                }
                double r = fabs(acc - rhs[n]);
                if (r > rmax) rmax = r;
                if (fabs(rhs[n]) > smax) smax = fabs(rhs[n]);
            }
    if (scale) *scale = smax;
    return rmax;
}

/* One red-black SOR sweep (Sec. II: SOR for the Poisson equation): red
 * nodes ((x + y + z) even) first, each set to the over-relaxed solution of
 * its own equation; Dirichlet nodes keep their potential. */
static void sor_sweep(const ora_state *s, const double *eps, const double *rhs, double *phi,
                      double omega) {
    for (int colour = 0; colour < 2; ++colour) {
#pragma omp parallel for schedule(static)
        for (int z = 0; z < s->P.nz; ++z)
            for (int y = 0; y < s->P.ny; ++y)
                for (int x = 0; x < s->P.nx; ++x) {
                    if (((x + y + z) & 1) != colour) continue;
                    int64_t n = node_index(s, x, y, z);
                    if (s->type[n] & T_DIRICHLET) continue;
                    double A = 0.0, B = 0.0;
                    for (int f = 0; f < 6; ++f) {
                        int64_t m = neighbour(s, x, y, z, FACE[f][0], FACE[f][1], FACE[f][2]);
                        if (m < 0) continue;
                        double ef = 0.5 * (eps[n] + eps[m]);
                        A += ef;
                        B += ef * phi[m];
                    }
                    phi[n] = (1.0 - omega) * phi[n] + omega * (B - rhs[n]) / A;
                }
    }
}

/* Zero-mean gauge of a domain without Dirichlet nodes (the periodic problem
 * fixes phi only up to a constant). */
static void gauge(const ora_state *s, double *phi) {
    if (s->has_dirichlet) return;
    nsum m = {0, 0};
    for (int64_t n = 0; n < s->N; ++n) ns_add(&m, phi[n]);
    double mean = ns_val(&m) / (double)s->N;
    for (int64_t n = 0; n < s->N; ++n) phi[n] -= mean;
}

/* Red-black SOR with a stop rule: at most `sweeps` sweeps; with tol > 0 the
 * residual is checked after every `check_every` sweeps (0: only after the
 * last) and the sweeps end once it is at most tol * max|rhs|.  The residual
 * after the last sweep done goes to *res, max|rhs| to *scale, the sweeps
 * done are returned; then the gauge.  Residuals are taken before the gauge
 * (they do not depend on it). */
int ora_poisson_solve(const ora_state *s, const double *eps, const double *rhs, double *phi,
                      int sweeps, double omega, double tol, int check_every, double *res,
                      double *scale) {
    int done = 0;
    double r = 0.0, sc = 0.0;
    int have = 0;
    while (done < sweeps) {
        sor_sweep(s, eps, rhs, phi, omega);
        ++done;
        have = 0;
        if (tol > 0.0 && check_every > 0 && done % check_every == 0 && done < sweeps) {
            r = ora_poisson_residual(s, eps, rhs, phi, &sc);
            have = 1;
            if (r <= tol * sc) break;
        }
    }
    if (!have) r = ora_poisson_residual(s, eps, rhs, phi, &sc);
    gauge(s, phi);
    if (res) *res = r;
    if (scale) *scale = sc;
    return done;
}

/* Exactly `sweeps` sweeps (then the gauge), for the solver pins. */
void ora_poisson(const ora_state *s, const double *eps, const double *rhs, double *phi,
                 int sweeps, double omega) {
    for (int sw = 0; sw < sweeps; ++sw) sor_sweep(s, eps, rhs, phi, omega);
    gauge(s, phi);
}

static void poisson(ora_state *s) {
    const int64_t N = s->N;
    double *eps = (double *)malloc(N * sizeof(double));
    for (int64_t n = 0; n < N; ++n) eps[n] = 1.0 + s->rho[n];
    s->qbar = ora_poisson_rhs(s, eps, s->q, s->rhs);
    s->sor_done = ora_poisson_solve(s, eps, s->rhs, s->phi, s->P.sor_sweeps, s->P.sor_omega,
                                    s->P.sor_tol, s->P.sor_check_every, &s->sor_res, &s->sor_scale);
    if (s->P.sor_tol > 0.0 && !(s->sor_res <= s->P.sor_tol * s->sor_scale)) s->sor_noconv++;
    free(eps);
}

/* E = E_ext - grad phi (19-point gradient), |E|^2, and the electric body
 * force F_el = q E + (eps - 1)/2 grad |E|^2 (Eq. force_el2; with the
 * electrostriction switch off, F_el = q E as in the text after Eq. add). */
static void electric(ora_state *s) {
    const int64_t N = s->N;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < s->P.nz; ++z)
        for (int y = 0; y < s->P.ny; ++y)
            for (int x = 0; x < s->P.nx; ++x) {
                int64_t n = node_index(s, x, y, z);
                double g[3];
                gradient19(s, s->phi, x, y, z, 1, g);
                double e0 = s->P.E_ext[0] - g[0], e1 = s->P.E_ext[1] - g[1], e2 = s->P.E_ext[2] - g[2];
                s->E[n] = e0; s->E[N + n] = e1; s->E[2 * N + n] = e2;
                s->E2[n] = e0 * e0 + e1 * e1 + e2 * e2;
            }
#pragma omp parallel for schedule(static)
    for (int z = 0; z < s->P.nz; ++z)
        for (int y = 0; y < s->P.ny; ++y)
            for (int x = 0; x < s->P.nx; ++x) {
                int64_t n = node_index(s, x, y, z);
                double F[3] = {0, 0, 0};
                if (kind(s, n) == T_FLUID) {
                    for (int a = 0; a < 3; ++a) F[a] = s->q[n] * s->E[a * N + n];
                    if (s->P.electrostriction) {
                        double g[3];
                        gradient19(s, s->E2, x, y, z, 1, g);
                        for (int a = 0; a < 3; ++a) F[a] += 0.5 * s->rho[n] * g[a];
                    }
                }
                for (int a = 0; a < 3; ++a) s->Fel[a * N + n] = F[a];
            }
}

/* Shan-Chen interaction (Eq. sc), generalised to components sigma, sigma':
 *   F^s = -psi^s(r) sum_s' G_ss' sum_{p: r+c_p fluid} w_p psi^s'(r+c_p) c_p
 *         - psi^s(r) sum_s' Gw_ss' sum_{p: r+c_p wall} w_p psi^s'(r) c_p:
 * a wall neighbour carries the node's own psi, weighted by the fluid-wall
 * couplings (one component: the printed form; Gw = G: no net wall force on a
 * uniform fluid),
 * psi = 1 - exp(-rho) (rho_0 = 1).  The electric force is shared among the
 * components by mass fraction.  Total F^s = F_int^s + F_el^s. */
static void forces(ora_state *s) {
    LAT_LOCALS(s);
    const int64_t N = s->N;
    const int C = s->C;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < s->P.nz; ++z)
        for (int y = 0; y < s->P.ny; ++y)
            for (int x = 0; x < s->P.nx; ++x) {
                int64_t n = node_index(s, x, y, z);
                if (kind(s, n) != T_FLUID) {
                    for (int sg = 0; sg < C; ++sg)
                        for (int a = 0; a < 3; ++a) s->F[((int64_t)sg * 3 + a) * N + n] = 0.0;
                    continue;
                }
                double rt = 0.0;
                for (int sg = 0; sg < C; ++sg) rt += s->rho[(int64_t)sg * N + n];
                for (int sg = 0; sg < C; ++sg) {
                    double acc[3] = {0, 0, 0}, wall[3] = {0, 0, 0};
                    for (int p = 1; p < Q; ++p) {
                        int64_t m = neighbour(s, x, y, z, CV[p][0], CV[p][1], CV[p][2]);
                        if (is_solid(s, m)) {
                            for (int a = 0; a < 3; ++a) wall[a] += WV[p] * CV[p][a];
                            continue;
                        }
                        double sp = 0.0;
                        for (int t = 0; t < C; ++t) sp += s->P.G[sg][t] * s->psi[(int64_t)t * N + m];
                        for (int a = 0; a < 3; ++a) acc[a] += WV[p] * sp * CV[p][a];
                    }
                    double ps = s->psi[(int64_t)sg * N + n];
                    double gw = 0.0;
                    for (int t = 0; t < C; ++t) gw += s->P.Gw[sg][t] * s->psi[(int64_t)t * N + n];
                    double frac = s->rho[(int64_t)sg * N + n] / rt;
                    for (int a = 0; a < 3; ++a) {
                        double Fi = -ps * acc[a] - ps * gw * wall[a];
                        s->F[((int64_t)sg * 3 + a) * N + n] = Fi + frac * s->Fel[a * N + n];
                    }
                }
            }
}

/* Velocity inlet (the jet set-up of Sec. III.B: Poiseuille velocity at the
 * inlet nodes, density that of the liquid).  After each step's moments an
 * inlet node holds, per component,
 *   inlet_mode 0: f_eq(rho_nb, u_bc), rho_nb the w-weighted mean density of
 *     its fluid neighbours, sum_p w_p rho(r + c_p) / sum_p w_p (rho_in when it
 *     has none);
 *   inlet_mode 1 + a: f_eq(rho_in, ubar u_bc), the profile u_bc rescaled by
 *     the mean velocity measured inside the nozzle in the same step (the
 *     paper's inlet). */
static void inlet_populations(const ora_state *s, int x, int y, int z, int sg, double *out) {
    LAT_LOCALS(s);
    const int64_t N = s->N;
    const int64_t n = node_index(s, x, y, z);
    if (s->P.inlet_mode > 0) {
        double u[3] = {s->ubar * s->u_bc[n], s->ubar * s->u_bc[N + n], s->ubar * s->u_bc[2 * N + n]};
        feq_lat(s->lat, s->P.rho_in[sg], u, out);
        return;
    }
    double sw = 0.0, sr = 0.0;
    for (int p = 1; p < Q; ++p) {
        int64_t m = neighbour(s, x, y, z, CV[p][0], CV[p][1], CV[p][2]);
        if (m < 0 || kind(s, m) != T_FLUID) continue;
        sw += WV[p];
        sr += WV[p] * s->rho[(int64_t)sg * N + m];
    }
    double u[3] = {s->u_bc[n], s->u_bc[N + n], s->u_bc[2 * N + n]};
    feq_lat(s->lat, sw > 0.0 ? sr / sw : s->P.rho_in[sg], u, out);
}

/* Collision (Eq. lattice-b) with alpha (Eq. entropic), beta from the
 * Newtonian or Carreau viscosity (Eqs. strain, stress, strain2, carreau,
 * beta) and the exact-difference source S = f_eq(rho, u + F/rho) - f_eq(rho, u)
 * (Eq. add).  Each component relaxes to the equilibrium at its own
 * velocity j/rho. */
static void collide(ora_state *s) {
    LAT_LOCALS(s);
    const int64_t N = s->N;
    const int C = s->C;
    int64_t nfb = 0, nnf = 0, nneg = 0;
#pragma omp parallel for schedule(static) reduction(+ : nfb, nnf, nneg)
    for (int z = 0; z < s->P.nz; ++z)
        for (int y = 0; y < s->P.ny; ++y)
            for (int x = 0; x < s->P.nx; ++x) {
                int64_t n = node_index(s, x, y, z);
                int k = kind(s, n);
                double rt = 0.0, mom[3] = {0, 0, 0};
                for (int sg = 0; sg < C; ++sg) {
                    double r = s->rho[(int64_t)sg * N + n];
                    rt += r;
                    for (int a = 0; a < 3; ++a)
                        mom[a] += s->jm[((int64_t)sg * 3 + a) * N + n] +
                                  0.5 * s->F[((int64_t)sg * 3 + a) * N + n];
                }
                for (int a = 0; a < 3; ++a) s->uph[a * N + n] = (k == T_SOLID) ? 0.0 : mom[a] / rt;
                for (int sg = 0; sg < C; ++sg) {
                    double *fo = s->fn + (int64_t)sg * Q * N;
                    if (k != T_FLUID) {
                        /* outlet and solid nodes keep their populations; inlet nodes are reset */
                        const double *fs = s->f + (int64_t)sg * Q * N;
                        if (k == T_INLET) {
                            double fi[QMAX];
                            inlet_populations(s, x, y, z, sg, fi);
                            for (int p = 0; p < Q; ++p) fo[p * N + n] = fi[p];
                        } else {
                            for (int p = 0; p < Q; ++p) fo[p * N + n] = fs[p * N + n];
                        }
                        s->alpha[(int64_t)sg * N + n] = 0.0;
                        s->iters[(int64_t)sg * N + n] = 0;
                        s->nu[(int64_t)sg * N + n] = 0.0;
                        continue;
                    }
                    double f[QMAX], fe[QMAX], u[3];
                    const double *fp = s->fp + (int64_t)sg * Q * N;
                    for (int p = 0; p < Q; ++p) f[p] = fp[p * N + n];
                    double r = s->rho[(int64_t)sg * N + n];
                    for (int a = 0; a < 3; ++a) u[a] = s->jm[((int64_t)sg * 3 + a) * N + n] / r;
                    feq_lat(s->lat, r, u, fe);
                    int its;
                    double al = alpha_lat(s->lat, f, fe, r, 2.0, s->P.newton_rtol, s->P.newton_max, &its);
                    if (its < 0) nfb++;
                    s->alpha[(int64_t)sg * N + n] = al;
                    s->iters[(int64_t)sg * N + n] = its;
                    double nu = s->P.nu0;
                    if (s->P.carreau) {
                        double Pi[6] = {0, 0, 0, 0, 0, 0};
                        for (int p = 0; p < Q; ++p) {
                            double d = f[p] - fe[p];
                            Pi[0] += d * CV[p][0] * CV[p][0];
                            Pi[1] += d * CV[p][1] * CV[p][1];
                            Pi[2] += d * CV[p][2] * CV[p][2];
                            Pi[3] += d * CV[p][0] * CV[p][1];
                            Pi[4] += d * CV[p][0] * CV[p][2];
                            Pi[5] += d * CV[p][1] * CV[p][2];
                        }
                        double Pn = ora_sym3_norm2(Pi);
                        double gd = ora_shear_rate(Pn, r, al, s->P.nu0, s->P.nu_inf, s->P.lam,
                                                   s->P.n_flow);
                        nu = ora_carreau_nu(gd, s->P.nu0, s->P.nu_inf, s->P.lam, s->P.n_flow);
                    }
                    s->nu[(int64_t)sg * N + n] = nu;
                    double beta = CS2 / (2.0 * nu + CS2);
                    double u2[3], fe2[QMAX];
                    for (int a = 0; a < 3; ++a) u2[a] = u[a] + s->F[((int64_t)sg * 3 + a) * N + n] / r;
                    feq_lat(s->lat, r, u2, fe2);
                    for (int p = 0; p < Q; ++p) {
                        double v = f[p] + al * beta * (fe[p] - f[p]) + (fe2[p] - fe[p]);
                        if (!isfinite(v)) nnf++;
                        else if (v < 0.0) nneg++;
                        fo[p * N + n] = v;
                    }
                }
            }
    s->nfallback += nfb;
    s->nerr_nonfinite += nnf;
    s->nerr_negative += nneg;
    double *t = s->f; s->f = s->fn; s->fn = t;
}

void ora_step(ora_state *s, int nsteps) {
    for (int it = 0; it < nsteps; ++it) {
        stream_and_moments(s);
        interface_fields(s);
        charge(s);
        poisson(s);
        electric(s);
        forces(s);
        collide(s);
    }
}

/* ------------------------------------------------------------ access */
enum {
    F_RHO = 0, F_J, F_PSI, F_GRAD, F_NHAT, F_K, F_BULK, F_SURF, F_Q, F_PHI, F_RHS, F_E, F_E2,
    F_FEL, F_F, F_ALPHA, F_NU, F_UPH, F_POP, F_PULLED
};

/* Copies a stored field into out; returns the number of doubles written. */
int64_t ora_field(const ora_state *s, int which, double *out) {
    LAT_LOCALS(s);
    int64_t N = s->N, C = s->C;
    const double *src = NULL;
    int64_t cnt = 0;
    switch (which) {
    case F_RHO: src = s->rho; cnt = C * N; break;
    case F_J: src = s->jm; cnt = C * 3 * N; break;
    case F_PSI: src = s->psi; cnt = C * N; break;
    case F_GRAD: src = s->grad; cnt = 3 * N; break;
    case F_NHAT: src = s->nhat; cnt = 3 * N; break;
    case F_K: src = s->K; cnt = N; break;
    case F_BULK: src = s->bulk; cnt = N; break;
    case F_SURF: src = s->surf; cnt = N; break;
    case F_Q: src = s->q; cnt = N; break;
    case F_PHI: src = s->phi; cnt = N; break;
    case F_RHS: src = s->rhs; cnt = N; break;
    case F_E: src = s->E; cnt = 3 * N; break;
    case F_E2: src = s->E2; cnt = N; break;
    case F_FEL: src = s->Fel; cnt = 3 * N; break;
    case F_F: src = s->F; cnt = C * 3 * N; break;
    case F_ALPHA: src = s->alpha; cnt = C * N; break;
    case F_NU: src = s->nu; cnt = C * N; break;
    case F_UPH: src = s->uph; cnt = 3 * N; break;
    case F_POP: src = s->f; cnt = C * Q * N; break;
    case F_PULLED: src = s->fp; cnt = C * Q * N; break;
    default: return -1;
    }
    memcpy(out, src, cnt * sizeof(double));
    return cnt;
}

void ora_iters(const ora_state *s, int32_t *out) { memcpy(out, s->iters, s->C * s->N * sizeof(int32_t)); }

void ora_set_populations(ora_state *s, const double *f) {
    LAT_LOCALS(s);
    memcpy(s->f, f, (size_t)s->C * Q * s->N * sizeof(double));
}
void ora_set_phi(ora_state *s, const double *phi) { memcpy(s->phi, phi, s->N * sizeof(double)); }

/* counters: fallbacks, non-finite and negative post-collision populations,
 * plus the two charge integrals and the neutralising charge of the last step */
void ora_counters(const ora_state *s, int64_t out_i[3], double out_d[3]) {
    out_i[0] = s->nfallback; out_i[1] = s->nerr_nonfinite; out_i[2] = s->nerr_negative;
    out_d[0] = s->Sb; out_d[1] = s->Ss; out_d[2] = s->qbar;
}

/* Poisson solve of the last step: residual and its scale max|rhs|, sweeps
 * done, and the steps whose solve missed the tolerance so far. */
void ora_poisson_stats(const ora_state *s, double out_d[2], int64_t out_i[2]) {
    out_d[0] = s->sor_res; out_d[1] = s->sor_scale;
    out_i[0] = s->sor_done; out_i[1] = s->sor_noconv;
}

/* Mean velocity inside the nozzle measured in the last step (inlet_mode > 0). */
double ora_inlet_ubar(const ora_state *s) { return s->ubar; }

/* Lattice tables (for the tests): D3Q19. */
void ora_lattice(int32_t c[19 * 3], double w[19]) {
    for (int p = 0; p < 19; ++p) {
        for (int a = 0; a < 3; ++a) c[p * 3 + a] = LAT_D3Q19.c[p][a];
        w[p] = LAT_D3Q19.w[p];
    }
}
/* Tables of lattice `lattice` (0 D3Q19, 1 D2Q9); returns its Q. */
int ora_lattice_q(int lattice, int32_t *c, double *w) {
    const ora_lat *L = lattice_of(lattice);
    for (int p = 0; p < L->q; ++p) {
        for (int a = 0; a < 3; ++a) c[p * 3 + a] = L->c[p][a];
        w[p] = L->w[p];
    }
    return L->q;
}

int ora_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
