/*
 * dugks_oracle.c -- plain FP64 CPU oracle of one incompressible-DUGKS step
 * with body force (arXiv:1411.6121).
 *
 * TEST INFRASTRUCTURE ONLY: used by the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg.  It is deliberately plain: scalar loops over
 * cell centres and interfaces, FP64, every quantity of an interface
 * (cross-point values, gradient, wall rule, moments, original distribution,
 * flux) recomputed where it is used, no blocking or fusion across points.
 * It shares no code with the HIP path.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (see build.py).
 * Every loop over points writes disjoint outputs in a fixed per-point
 * operation order, so results do not depend on the thread count.
 *
 * Every public function is pinned by tests/test_oracle_*.py to what the
 * paper and the mathematics fix (printed tables, closed forms, invariants,
 * analytic flows, finite differences), never to the HIP path.
 */
#include "dugks_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXQ 27

/* ------------------------------------------------------------------------ */
/* derived context                                                           */
/* ------------------------------------------------------------------------ */
typedef struct {
    int D, Q;
    int e[MAXQ][3];
    double W[MAXQ];
    int opp[MAXQ];
    double c;              /* c = sqrt(3 RT)                               */
    double xi[MAXQ][3];    /* xi_q = c e_q                                 */
    int n[3];              /* cells per axis (1 for the absent z in 2-D)    */
    int E[3];              /* extended extent: n+2 on active axes, else 1   */
    int off[3];            /* 1 on active axes (ghost layer), else 0        */
    int per[3];            /* periodic flag per active axis                 */
    double *X[3];          /* face coordinates X_0..X_n                     */
    double *xc[3];         /* centre coordinates x_{-1}..x_n (offset +1)    */
    double *w[3];          /* face f: weight of the right cell, f = 0..n    */
    double *g[3];          /* face f: 1/(x_f - x_{f-1}), f = 0..n           */
    double *dl[3];         /* cell widths Delta_i, i = 0..n-1               */
    double rlo[3], rhi[3]; /* ghost extrapolation ratios (wall axes)        */
} octx;

static void ctx_free(octx* o)
{
    for (int a = 0; a < 3; ++a) {
        free(o->X[a]); free(o->xc[a]); free(o->w[a]); free(o->g[a]); free(o->dl[a]);
        o->X[a] = o->xc[a] = o->w[a] = o->g[a] = o->dl[a] = NULL;
    }
}

/* Velocity set, Sec. II.C.  One-dimensional three-point Gauss-Hermite rule:
 * abscissae sqrt(3RT){-1,0,1}; the weights are 2/3 at 0 and 1/6 at +-1
 * (the printed 1/3 is a misprint: the printed D2Q9 and D3Q27 weights are
 * products of 2/3 and 1/6, and the weights must sum to one).
 * D2Q9 is the tensor product in the paper's order (e_x outer, e_y inner).
 * D3Q27 is the paper's 3-D set (Sec. II.C): the full tensor product, e_x
 * outer, e_y, e_z inner, weights products of the 1-D weights.
 * D3Q19 (not in the paper) keeps the same order and drops the eight
 * |e|^2 = 3 corners, with weights 1/3, 1/18, 1/36. */
static int make_lattice(int lattice, int e[MAXQ][3], double W[MAXQ], int opp[MAXQ])
{
    int Q = 0;
    if (lattice == 9) {
        const double w1[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};
        for (int ex = -1; ex <= 1; ++ex)
            for (int ey = -1; ey <= 1; ++ey) {
                e[Q][0] = ex; e[Q][1] = ey; e[Q][2] = 0;
                W[Q] = w1[ex + 1] * w1[ey + 1];
                ++Q;
            }
    } else if (lattice == 19) {
        for (int ex = -1; ex <= 1; ++ex)
            for (int ey = -1; ey <= 1; ++ey)
                for (int ez = -1; ez <= 1; ++ez) {
                    int m = ex * ex + ey * ey + ez * ez;
                    if (m == 3) continue;
                    e[Q][0] = ex; e[Q][1] = ey; e[Q][2] = ez;
                    W[Q] = (m == 0) ? 1.0 / 3.0 : (m == 1) ? 1.0 / 18.0 : 1.0 / 36.0;
                    ++Q;
                }
    } else if (lattice == 27) {
        const double w1[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};
        for (int ex = -1; ex <= 1; ++ex)
            for (int ey = -1; ey <= 1; ++ey)
                for (int ez = -1; ez <= 1; ++ez) {
                    e[Q][0] = ex; e[Q][1] = ey; e[Q][2] = ez;
                    W[Q] = w1[ex + 1] * w1[ey + 1] * w1[ez + 1];
                    ++Q;
                }
    } else {
        return -1;
    }
    for (int q = 0; q < Q; ++q) {
        opp[q] = -1;
        for (int r = 0; r < Q; ++r)
            if (e[r][0] == -e[q][0] && e[r][1] == -e[q][1] && e[r][2] == -e[q][2]) opp[q] = r;
    }
    return Q;
}

/* face coordinates of one axis: uniform, the tanh stretching of
 * Eq. (Nonuniform_mesh): zeta_i = 1/2 + tanh(k(i/N - 1/2)) / (2 tanh(k/2)),
 * or given coordinates (0 = X_0 < ... < X_N = L); -1 if those are not
 * strictly increasing from 0 to L */
static int make_faces(const oracle_cfg* cfg, int a, int N, double L, double* X)
{
    const int kind = cfg->mesh[a];
    if (kind == OR_CUSTOM) {
        const double* F = cfg->faces[a];
        if (!F || F[0] != 0.0 || F[N] != L) return -1;
        for (int i = 0; i <= N; ++i) X[i] = F[i];
        for (int i = 0; i < N; ++i)
            if (!(X[i + 1] > X[i])) return -1;
        return 0;
    }
    for (int i = 0; i <= N; ++i) {
        if (kind == OR_TANH) {
            double zeta = 0.5 + tanh(cfg->k_stretch * ((double)i / N - 0.5)) / (2.0 * tanh(0.5 * cfg->k_stretch));
            X[i] = L * zeta;
        } else {
            X[i] = L * (double)i / N;
        }
    }
    X[0] = 0.0;
    X[N] = L;
    return 0;
}

static int setup(octx* o, const oracle_cfg* cfg)
{
    memset(o, 0, sizeof(*o));
    o->Q = make_lattice(cfg->lattice, o->e, o->W, o->opp);
    if (o->Q < 0) return -1;
    o->D = (cfg->lattice == 9) ? 2 : 3;
    if (!(cfg->RT > 0) || !(cfg->tau > 0) || !(cfg->dt > 0) || !(cfg->rho0 > 0)) return -1;
    if (cfg->model != 0 && cfg->model != 1) return -1;
    o->c = sqrt(3.0 * cfg->RT);
    for (int q = 0; q < o->Q; ++q)
        for (int a = 0; a < 3; ++a) o->xi[q][a] = o->c * o->e[q][a];
    for (int a = 0; a < 3; ++a) {
        if (a < o->D) {
            o->n[a] = cfg->n[a];
            o->E[a] = cfg->n[a] + 2;
            o->off[a] = 1;
            int lo = cfg->bc[2 * a], hi = cfg->bc[2 * a + 1];
            if ((lo == OR_PERIODIC) != (hi == OR_PERIODIC)) return -1;
            o->per[a] = (lo == OR_PERIODIC);
            if (o->n[a] < (o->per[a] ? 1 : 2)) return -1;
        } else {
            o->n[a] = 1; o->E[a] = 1; o->off[a] = 0; o->per[a] = 1;
        }
    }
    for (int a = 0; a < o->D; ++a) {
        int N = o->n[a];
        double L = cfg->L[a];
        if (!(L > 0)) { ctx_free(o); return -1; }
        o->X[a] = (double*)malloc(sizeof(double) * (N + 1));
        o->xc[a] = (double*)malloc(sizeof(double) * (N + 2));
        o->w[a] = (double*)malloc(sizeof(double) * (N + 1));
        o->g[a] = (double*)malloc(sizeof(double) * (N + 1));
        o->dl[a] = (double*)malloc(sizeof(double) * N);
        if (make_faces(cfg, a, N, L, o->X[a])) { ctx_free(o); return -1; }
        double* X = o->X[a];
        double* xc = o->xc[a] + 1; /* xc[-1..N] */
        for (int i = 0; i < N; ++i) {
            xc[i] = 0.5 * (X[i] + X[i + 1]);
            o->dl[a][i] = X[i + 1] - X[i];
        }
        if (o->per[a]) {           /* wrapped neighbours, shifted by L */
            xc[-1] = xc[N - 1] - L;
            xc[N] = xc[0] + L;
        } else {                   /* ghost centres mirrored in the wall */
            xc[-1] = 2.0 * X[0] - xc[0];
            xc[N] = 2.0 * X[N] - xc[N - 1];
        }
        /* face f lies between cells f-1 and f */
        for (int f = 0; f <= N; ++f) {
            o->w[a][f] = (X[f] - xc[f - 1]) / (xc[f] - xc[f - 1]);
            o->g[a][f] = 1.0 / (xc[f] - xc[f - 1]);
        }
        if (o->per[a]) { /* face N is face 0 */
            o->w[a][N] = o->w[a][0];
            o->g[a][N] = o->g[a][0];
        } else {
            o->rlo[a] = (xc[-1] - xc[0]) / (xc[1] - xc[0]);
            o->rhi[a] = (xc[N] - xc[N - 1]) / (xc[N - 2] - xc[N - 1]);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* point-local formulas                                                      */
/* ------------------------------------------------------------------------ */

/* Eq. (icfeq): W_q { rho + rho0 [ xi.u/RT + (xi.u)^2/(2 RT^2) - |u|^2/(2 RT) ] }
 * (model 0), or the original Eq. (feq):
 *   W_q rho [ 1 + xi.u/RT + (xi.u)^2/(2 RT^2) - |u|^2/(2 RT) ]      (model 1) */
static double feq_q(const octx* o, const oracle_cfg* cfg, int q, double rho, const double* u)
{
    double RT = cfg->RT, xu = 0.0, uu = 0.0;
    for (int a = 0; a < o->D; ++a) { xu += o->xi[q][a] * u[a]; uu += u[a] * u[a]; }
    const double poly = xu / RT + xu * xu / (2.0 * RT * RT) - uu / (2.0 * RT);
    if (cfg->model == 1) return o->W[q] * rho * (1.0 + poly);
    return o->W[q] * (rho + cfg->rho0 * poly);
}

/* density that multiplies u in the momentum of the model: rho0 in
 * Eq. (macro_values) (model 0), rho in the original model's
 * rho u = sum xi f + rho G dt/2 (model 1) */
static double mom_density(const oracle_cfg* cfg, double rho) { return cfg->model == 1 ? rho : cfg->rho0; }

/* Eq. (S), evaluated with the discrete equilibrium of the model in use (the
 * incompressible one, Eq. (icfeq), for model 0): S = G.(xi - u)/RT feq */
static double src_q(const octx* o, const oracle_cfg* cfg, int q, double rho, const double* u,
                    const double* G)
{
    double gx = 0.0;
    for (int a = 0; a < o->D; ++a) gx += G[a] * (o->xi[q][a] - u[a]);
    return gx / cfg->RT * feq_q(o, cfg, q, rho, u);
}

static double gtime(const oracle_cfg* cfg, double t) { return cos(cfg->omega * t + cfg->phase); }

/* ------------------------------------------------------------------------ */
/* indexing                                                                  */
/* ------------------------------------------------------------------------ */
static inline long cell_ext(const octx* o, int i, int j, int k)
{
    return ((long)(k + o->off[2]) * o->E[1] + (j + o->off[1])) * o->E[0] + (i + o->off[0]);
}
static inline long cell_int(const octx* o, int i, int j, int k)
{
    return ((long)k * o->n[1] + j) * o->n[0] + i;
}
static inline long ncells(const octx* o) { return (long)o->n[0] * o->n[1] * o->n[2]; }
static inline long ncells_ext(const octx* o) { return (long)o->E[0] * o->E[1] * o->E[2]; }

/* face point of axis a: coordinate c[a] in [0, n_a], others in [0, n_b) */
static inline long face_dim(const octx* o, int a, int b) { return b == a ? o->n[b] + 1 : o->n[b]; }
static inline long face_idx(const octx* o, int a, const int* c)
{
    return ((long)c[2] * face_dim(o, a, 1) + c[1]) * face_dim(o, a, 0) + c[0];
}
static inline long face_count(const octx* o, int a)
{
    return face_dim(o, a, 0) * face_dim(o, a, 1) * face_dim(o, a, 2);
}
/* cross point of the axis pair {a, b}: c[a] in [0,n_a], c[b] in [0,n_b] */
static inline long edge_dim(const octx* o, int a, int b, int d)
{
    return (d == a || d == b) ? o->n[d] + 1 : o->n[d];
}
static inline long edge_idx(const octx* o, int a, int b, const int* c)
{
    return ((long)c[2] * edge_dim(o, a, b, 1) + c[1]) * edge_dim(o, a, b, 0) + c[0];
}
static inline long edge_count(const octx* o, int a, int b)
{
    return edge_dim(o, a, b, 0) * edge_dim(o, a, b, 1) * edge_dim(o, a, b, 2);
}
static inline int pair_id(int a, int b) /* 0:{0,1} 1:{0,2} 2:{1,2} */
{
    if (a > b) { int t = a; a = b; b = t; }
    return (a == 0) ? (b == 1 ? 0 : 1) : 2;
}

/* Ghost layer of the extended cell set, for any field with ncomp values per
 * point.
 * Wall axes: linear extrapolation through the two nearest centres to the
 * mirrored ghost centre; periodic axes: copy of the wrapped cell.  Axes are
 * treated one after another over the growing extended range, so edge and
 * corner ghosts are tensor-product extrapolations. */
static void ghost_fill(const octx* o, double* v, int ncomp)
{
    for (int a = 0; a < o->D; ++a) {
        int lo[3], hi[3];
        for (int b = 0; b < 3; ++b) {
            if (b >= o->D) { lo[b] = 0; hi[b] = 0; continue; }
            if (b < a) { lo[b] = -1; hi[b] = o->n[b]; }
            else { lo[b] = 0; hi[b] = o->n[b] - 1; }
        }
        int N = o->n[a];
        for (int side = 0; side < 2; ++side) {
            int gc = side ? N : -1;
            lo[a] = hi[a] = gc;
            for (int k = lo[2]; k <= hi[2]; ++k)
                for (int j = lo[1]; j <= hi[1]; ++j)
                    for (int i = lo[0]; i <= hi[0]; ++i) {
                        int c[3] = {i, j, k};
                        int c0[3] = {i, j, k}, c1[3] = {i, j, k};
                        long dst = cell_ext(o, i, j, k);
                        if (o->per[a]) {
                            c0[a] = side ? 0 : N - 1;
                            long src = cell_ext(o, c0[0], c0[1], c0[2]);
                            for (int m = 0; m < ncomp; ++m) v[dst * ncomp + m] = v[src * ncomp + m];
                        } else {
                            double r = side ? o->rhi[a] : o->rlo[a];
                            c0[a] = side ? N - 1 : 0;
                            c1[a] = side ? N - 2 : 1;
                            long s0 = cell_ext(o, c0[0], c0[1], c0[2]);
                            long s1 = cell_ext(o, c1[0], c1[1], c1[2]);
                            for (int m = 0; m < ncomp; ++m)
                                v[dst * ncomp + m] = v[s0 * ncomp + m] + r * (v[s1 * ncomp + m] - v[s0 * ncomp + m]);
                        }
                        (void)c;
                    }
        }
    }
}

/* spatial force field G^ on the extended cell set (ghosts by step-2 rule) */
static double* force_ext(const octx* o, const double* force)
{
    if (!force) return NULL;
    const int D = o->D;
    long nc = ncells(o);
    double* G = (double*)calloc((size_t)ncells_ext(o) * D, sizeof(double));
    for (int k = 0; k < o->n[2]; ++k)
        for (int j = 0; j < o->n[1]; ++j)
            for (int i = 0; i < o->n[0]; ++i)
                for (int a = 0; a < D; ++a)
                    G[cell_ext(o, i, j, k) * D + a] = force[a * nc + cell_int(o, i, j, k)];
    ghost_fill(o, G, D);
    return G;
}

/* acceleration at a cell centre at time t */
static void accel_cell(const octx* o, const oracle_cfg* cfg, const double* Gext, long ce,
                       double gt, double* G)
{
    for (int a = 0; a < 3; ++a) G[a] = 0.0;
    for (int a = 0; a < o->D; ++a) G[a] = gt * (cfg->G[a] + (Gext ? Gext[ce * o->D + a] : 0.0));
}

/* acceleration at the face point of axis a with coords c, time factor gt:
 * the spatial part is interpolated between the two centres like f-bar-plus */
static void accel_face(const octx* o, const oracle_cfg* cfg, const double* Gext, int a,
                       const int* c, double gt, double* G)
{
    for (int d = 0; d < 3; ++d) G[d] = 0.0;
    int cl[3] = {c[0], c[1], c[2]}, cr[3] = {c[0], c[1], c[2]};
    cl[a] = c[a] - 1;
    double w = o->w[a][c[a]];
    long L = cell_ext(o, cl[0], cl[1], cl[2]), R = cell_ext(o, cr[0], cr[1], cr[2]);
    for (int d = 0; d < o->D; ++d) {
        double gh = 0.0;
        if (Gext) gh = (1.0 - w) * Gext[L * o->D + d] + w * Gext[R * o->D + d];
        G[d] = gt * (cfg->G[d] + gh);
    }
}

/* ------------------------------------------------------------------------ */
/* public: tables and point formulas                                         */
/* ------------------------------------------------------------------------ */
int oracle_lattice(int lattice, int* e, double* w)
{
    int E_[MAXQ][3], opp[MAXQ];
    double W[MAXQ];
    int Q = make_lattice(lattice, E_, W, opp);
    if (Q < 0) return -1;
    for (int q = 0; q < Q; ++q) {
        for (int a = 0; a < 3; ++a) e[q * 3 + a] = E_[q][a];
        w[q] = W[q];
    }
    return Q;
}

int oracle_mesh(const oracle_cfg* cfg, int axis, double* faces, double* centres)
{
    octx o;
    if (setup(&o, cfg)) return -1;
    if (axis < 0 || axis >= o.D) { ctx_free(&o); return -1; }
    int N = o.n[axis];
    for (int f = 0; f <= N; ++f) faces[f] = o.X[axis][f];
    for (int i = 0; i < N + 2; ++i) centres[i] = o.xc[axis][i];
    ctx_free(&o);
    return 0;
}

int oracle_feq(const oracle_cfg* cfg, double rho, const double* u, double* feq)
{
    octx o;
    if (setup(&o, cfg)) return -1;
    for (int q = 0; q < o.Q; ++q) feq[q] = feq_q(&o, cfg, q, rho, u);
    ctx_free(&o);
    return 0;
}

int oracle_force_term(const oracle_cfg* cfg, double rho, const double* u, const double* G,
                      double* S)
{
    octx o;
    if (setup(&o, cfg)) return -1;
    for (int q = 0; q < o.Q; ++q) S[q] = src_q(&o, cfg, q, rho, u, G);
    ctx_free(&o);
    return 0;
}

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* initialisation: f~0 = feq - dt/2 S (f = feq and Omega = 0 at equilibrium) */
/* ------------------------------------------------------------------------ */
int oracle_init(const oracle_cfg* cfg, const double* rho, const double* u, const double* force,
                double t0, double* f_out)
{
    octx o;
    if (setup(&o, cfg)) return -1;
    const int D = o.D, Q = o.Q;
    const long nc = ncells(&o);
    const double gt = gtime(cfg, t0);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < nc; ++c) {
        double r = rho ? rho[c] : cfg->rho0;
        double uu[3] = {0, 0, 0}, G[3] = {0, 0, 0};
        for (int a = 0; a < D; ++a) {
            if (u) uu[a] = u[a * nc + c];
            G[a] = gt * (cfg->G[a] + (force ? force[a * nc + c] : 0.0));
        }
        for (int q = 0; q < Q; ++q)
            f_out[q * nc + c] = feq_q(&o, cfg, q, r, uu) - 0.5 * cfg->dt * src_q(&o, cfg, q, r, uu, G);
    }
    ctx_free(&o);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* one time step t_n -> t_n + dt                                             */
/*                                                                           */
/* Written from the equations of Sec. II, organised around its three kinds  */
/* of work: a transform of every cell centre (Eqs. (macro_values),          */
/* (f_bar_+)) with the ghost layer of wall axes, a flux routine evaluated    */
/* once per interface (Eqs. (gradient), (BB)/(NEQ), (original_f),           */
/* (microflux)), and a conservative update of every cell                     */
/* (Eqs. (f_tilde_+), (evolution_equation)).                                 */
/* ------------------------------------------------------------------------ */

/* Density and velocity of one point from a distribution set, Eq.
 * (macro_values): rho = sum f, rho0 u = sum xi f + rho0 G dth (model 0), or
 * rho u = sum xi f + rho G dth (model 1).  dth is half the interval the
 * distribution is shifted by: dt/2 for f~ at centres, h/2 for f-bar at
 * interfaces. */
static void point_macro(const octx* o, const oracle_cfg* cfg, const double* f, const double* G, double dth,
                        double* rho, double* u)
{
    double r = 0.0, m[3] = {0, 0, 0};
    for (int q = 0; q < o->Q; ++q) {
        r += f[q];
        for (int a = 0; a < o->D; ++a) m[a] += o->xi[q][a] * f[q];
    }
    const double rm = mom_density(cfg, r);
    for (int a = 0; a < 3; ++a) u[a] = 0.0;
    for (int a = 0; a < o->D; ++a) u[a] = (m[a] + rm * G[a] * dth) / rm;
    *rho = r;
}

/* equilibrium (Eq. (icfeq), or Eq. (feq) for model 1) and force term
 * (Eq. (S)) of every velocity at one point */
static void point_eq(const octx* o, const oracle_cfg* cfg, double rho, const double* u, const double* G,
                     double* feq, double* S)
{
    for (int q = 0; q < o->Q; ++q) {
        feq[q] = feq_q(o, cfg, q, rho, u);
        double gx = 0.0;
        for (int a = 0; a < o->D; ++a) gx += G[a] * (o->xi[q][a] - u[a]);
        S[q] = gx / cfg->RT * feq[q];
    }
}

/* Eq. (f_bar_+) at every cell centre, from f~ at t_n with rho, u of
 * Eq. (macro_values) and G(x_c, t_n); then the ghost layer (extrapolated on
 * wall axes, wrapped on periodic ones).  phi is the extended cell array
 * [cell_ext][q]. */
static void transform_cells(const octx* o, const oracle_cfg* cfg, const double* fin, const double* Gext,
                            double gt, double* phi)
{
    const int Q = o->Q;
    const long nc = ncells(o);
    const double dt = cfg->dt, h = 0.5 * dt, tau = cfg->tau;
    const double a_f = (2.0 * tau - h) / (2.0 * tau + dt);
    const double a_eq = 3.0 * h / (2.0 * tau + dt);
    const double a_s = 3.0 * tau * h / (2.0 * tau + dt);
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < o->n[2]; ++k)
        for (int j = 0; j < o->n[1]; ++j)
            for (int i = 0; i < o->n[0]; ++i) {
                const long ci = cell_int(o, i, j, k), ce = cell_ext(o, i, j, k);
                double f[MAXQ], fe[MAXQ], S[MAXQ], G[3], rho, u[3];
                for (int q = 0; q < Q; ++q) f[q] = fin[q * nc + ci];
                accel_cell(o, cfg, Gext, ce, gt, G);
                point_macro(o, cfg, f, G, dt / 2.0, &rho, u);
                point_eq(o, cfg, rho, u, G, fe, S);
                for (int q = 0; q < Q; ++q) phi[ce * Q + q] = a_f * f[q] + a_eq * fe[q] + a_s * S[q];
            }
    ghost_fill(o, phi, Q);
}

/* The cross point of the interface of axis a with index c[a] and the
 * interface of axis b with index c[b] (c's other entry is a cell index):
 * its value is the bilinear interpolation of the 2 x 2 block of cells around
 * it, linear along a on the two rows (weight wa of the upper cell), then
 * linear along b (weight wb of the upper row).  cell[] receives the block in
 * the order (lower a, lower b), (upper a, lower b), (lower a, upper b),
 * (upper a, upper b). */
typedef struct {
    long cell[4];
    double wa, wb;
} ocross;

static void cross_point_at(const octx* o, int a, int b, const int* c, ocross* x)
{
    x->wa = o->w[a][c[a]];
    x->wb = o->w[b][c[b]];
    for (int m = 0; m < 4; ++m) {
        int cc[3] = {c[0], c[1], c[2]};
        if (!(m & 1)) cc[a] -= 1;
        if (!(m & 2)) cc[b] -= 1;
        x->cell[m] = cell_ext(o, cc[0], cc[1], cc[2]);
    }
}

static double cross_value(const octx* o, const double* phi, const ocross* x, int q)
{
    const int Q = o->Q;
    const double row_lo = (1.0 - x->wa) * phi[x->cell[0] * Q + q] + x->wa * phi[x->cell[1] * Q + q];
    const double row_hi = (1.0 - x->wa) * phi[x->cell[2] * Q + q] + x->wa * phi[x->cell[3] * Q + q];
    return (1.0 - x->wb) * row_lo + x->wb * row_hi;
}

/* Eqs. (interfaceEvof) and (gradient): f-bar(x_b, t_n + h) =
 * f-bar-plus(x_b) - h xi . sigma_b at the mid-point of the interface of axis
 * a with index c[a] (between cells c[a]-1 and c[a]).  f-bar-plus(x_b) is
 * linear interpolation between the two centres; the normal component of
 * sigma_b is their difference over their distance, a tangential component b
 * the difference of the cross-point values at the interface's two edges
 * along b over the interface width. */
static void interface_fbar(const octx* o, const double* phi, int a, const int* c, double h, double* fb)
{
    const int D = o->D, Q = o->Q;
    int cl[3] = {c[0], c[1], c[2]};
    cl[a] -= 1;
    const long L = cell_ext(o, cl[0], cl[1], cl[2]), R = cell_ext(o, c[0], c[1], c[2]);
    const double w = o->w[a][c[a]], gn = o->g[a][c[a]];
    ocross edge_lo[3], edge_hi[3];
    double inv_width[3] = {0, 0, 0};
    for (int b = 0; b < D; ++b) {
        if (b == a) continue;
        int c_up[3] = {c[0], c[1], c[2]};
        c_up[b] += 1;
        cross_point_at(o, a, b, c, &edge_lo[b]);
        cross_point_at(o, a, b, c_up, &edge_hi[b]);
        inv_width[b] = 1.0 / o->dl[b][c[b]];
    }
    for (int q = 0; q < Q; ++q) {
        double sig[3] = {0, 0, 0};
        sig[a] = gn * (phi[R * Q + q] - phi[L * Q + q]);
        for (int b = 0; b < D; ++b) {
            if (b == a) continue;
            sig[b] = (cross_value(o, phi, &edge_hi[b], q) - cross_value(o, phi, &edge_lo[b], q)) * inv_width[b];
        }
        double xs = 0.0;
        for (int b = 0; b < D; ++b) xs += o->xi[q][b] * sig[b];
        fb[q] = ((1.0 - w) * phi[L * Q + q] + w * phi[R * Q + q]) - h * xs;
    }
}

/* Density of the pressure condition on side s, from p = (rho - rho0) RT:
 * rho0 + p_w(t)/RT, where the wall pressure may follow the time factor g,
 * p_w(t) = pw + pw_osc g(t) (the oscillating inlet pressure of the
 * pressure-driven flow of Sec. III.C, Eq. (Wom_AS_Pressure)); g is taken at
 * the interface time t_n + h. */
static double pressure_wall_density(const oracle_cfg* cfg, int s, double g)
{
    return cfg->rho0 + (cfg->pw[s] + cfg->pw_osc[s] * g) / cfg->RT;
}

/* Wall interface of side s: the velocities entering the domain (xi.n < 0,
 * n the outward normal) are replaced by bounce-back, Eq. (BB) with
 * rho_w = rho0, or by non-equilibrium extrapolation, Eq. (NEQ), whose
 * non-equilibrium part is taken at x_c, the opposite interface of the same
 * wall cell (fo: f-bar there, rc/uc its moments).  Velocity condition:
 * (rho_alpha, u_alpha) = (rc, u_w); pressure condition: (rho0 + p_w/RT, uc)
 * with p_w at the interface time (time factor g).
 * The rules act on f-bar before its moments are taken. */
static void wall_condition(const octx* o, const oracle_cfg* cfg, int s, double* fw, const double* fo, double rc,
                           const double* uc, double g)
{
    const int D = o->D, Q = o->Q, a = s / 2;
    const int out = (s % 2) ? 1 : -1; /* outward normal along a */
    const double rho0 = cfg->rho0, RT = cfg->RT;
    if (cfg->bc[s] == OR_BOUNCE_BACK) {
        double before[MAXQ];
        for (int q = 0; q < Q; ++q) before[q] = fw[q];
        for (int q = 0; q < Q; ++q) {
            if (o->e[q][a] * out >= 0) continue;
            double xu = 0.0;
            for (int b = 0; b < D; ++b) xu += o->xi[q][b] * cfg->uw[s][b];
            fw[q] = before[o->opp[q]] + 2.0 * rho0 * o->W[q] * xu / RT;
        }
        return;
    }
    double ra, ua[3] = {0, 0, 0};
    if (cfg->bc[s] == OR_NEQ_VELOCITY) {
        ra = rc;
        for (int b = 0; b < D; ++b) ua[b] = cfg->uw[s][b];
    } else {
        ra = pressure_wall_density(cfg, s, g);
        for (int b = 0; b < D; ++b) ua[b] = uc[b];
    }
    for (int q = 0; q < Q; ++q) {
        if (o->e[q][a] * out >= 0) continue;
        fw[q] = feq_q(o, cfg, q, ra, ua) + (fo[q] - feq_q(o, cfg, q, rc, uc));
    }
}

/* Flux density xi_a f(x_b, t_n + h) of every velocity through the interface
 * of axis a with index c[a] (normal +e_a), the integrand of Eq. (microflux)
 * at the half step: f-bar from Eq. (gradient), the wall rule on wall
 * interfaces, the interface moments (macro_values with G(x_b, t_n + h) and
 * h/2), and f from f-bar by inverting Eq. (original_f):
 * f = 2 tau/(2 tau + h) f-bar + h/(2 tau + h) feq + tau h/(2 tau + h) S. */
static void interface_flux(const octx* o, const oracle_cfg* cfg, const double* phi, const double* Gext, double gth,
                           int a, const int* c, double* flux)
{
    const int Q = o->Q;
    const double h = 0.5 * cfg->dt, tau = cfg->tau;
    const double b_f = 2.0 * tau / (2.0 * tau + h);
    const double b_eq = h / (2.0 * tau + h);
    const double b_s = tau * h / (2.0 * tau + h);
    double fb[MAXQ], fe[MAXQ], S[MAXQ], G[3], rho, u[3];
    interface_fbar(o, phi, a, c, h, fb);
    const int N = o->n[a];
    if (!o->per[a] && (c[a] == 0 || c[a] == N)) {
        int co[3] = {c[0], c[1], c[2]};
        co[a] = (c[a] == 0) ? 1 : N - 1;
        double fo[MAXQ], Go[3], rc, uc[3];
        interface_fbar(o, phi, a, co, h, fo);
        accel_face(o, cfg, Gext, a, co, gth, Go);
        point_macro(o, cfg, fo, Go, h / 2.0, &rc, uc);
        wall_condition(o, cfg, 2 * a + (c[a] == N), fb, fo, rc, uc, gth);
    }
    accel_face(o, cfg, Gext, a, c, gth, G);
    point_macro(o, cfg, fb, G, h / 2.0, &rho, u);
    point_eq(o, cfg, rho, u, G, fe, S);
    for (int q = 0; q < Q; ++q) flux[q] = o->xi[q][a] * (b_f * fb[q] + b_eq * fe[q] + b_s * S[q]);
}

/* the step's work arrays, kept across the steps of one run */
typedef struct {
    double* phi;       /* f-bar-plus on the extended cell set */
    double* Gext;      /* spatial force on the extended cell set, or NULL */
    double* flux[3];   /* flux densities on the interfaces of each axis */
} oworkspace;

static int work_alloc(const octx* o, const double* force, oworkspace* w)
{
    memset(w, 0, sizeof(*w));
    w->phi = (double*)calloc((size_t)ncells_ext(o) * o->Q, sizeof(double));
    int ok = w->phi != NULL;
    for (int a = 0; a < o->D; ++a) {
        w->flux[a] = (double*)malloc(sizeof(double) * face_count(o, a) * o->Q);
        ok = ok && w->flux[a] != NULL;
    }
    w->Gext = force_ext(o, force);
    return ok ? 0 : -1;
}

static void work_free(oworkspace* w)
{
    free(w->phi);
    free(w->Gext);
    for (int a = 0; a < 3; ++a) free(w->flux[a]);
    memset(w, 0, sizeof(*w));
}

static void step_with(const octx* o, const oracle_cfg* cfg, oworkspace* w, const double* fin, double* fout,
                      double t)
{
    const int D = o->D, Q = o->Q;
    const long nc = ncells(o);
    const double dt = cfg->dt, h = 0.5 * dt;
    const double gt = gtime(cfg, t), gth = gtime(cfg, t + h);

    transform_cells(o, cfg, fin, w->Gext, gt, w->phi);

    for (int a = 0; a < D; ++a) {
        const int d0 = face_dim(o, a, 0), d1 = face_dim(o, a, 1), d2 = face_dim(o, a, 2);
#pragma omp parallel for collapse(2) schedule(static)
        for (int k = 0; k < d2; ++k)
            for (int j = 0; j < d1; ++j)
                for (int i = 0; i < d0; ++i) {
                    const int c[3] = {i, j, k};
                    interface_flux(o, cfg, w->phi, w->Gext, gth, a, c, w->flux[a] + face_idx(o, a, c) * Q);
                }
    }

    /* Eq. (evolution_equation) with f~+ of Eq. (f_tilde_+): the flux out of
     * cell V through its interfaces j is sum_j (xi.n_j) f s_j; on the
     * tensor mesh interface j of axis a has area s_a = |V| / Delta_a */
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < o->n[2]; ++k)
        for (int j = 0; j < o->n[1]; ++j)
            for (int i = 0; i < o->n[0]; ++i) {
                const int c[3] = {i, j, k};
                const long ci = cell_int(o, i, j, k), ce = cell_ext(o, i, j, k);
                double V = 1.0, s[3] = {1, 1, 1};
                for (int a = 0; a < D; ++a) V *= o->dl[a][c[a]];
                for (int a = 0; a < D; ++a)
                    for (int b = 0; b < D; ++b)
                        if (b != a) s[a] *= o->dl[b][c[b]];
                const double* up[3] = {NULL, NULL, NULL};
                const double* dn[3] = {NULL, NULL, NULL};
                for (int a = 0; a < D; ++a) {
                    int cp[3] = {i, j, k};
                    cp[a] += 1;
                    dn[a] = w->flux[a] + face_idx(o, a, c) * Q;
                    up[a] = w->flux[a] + face_idx(o, a, cp) * Q;
                }
                for (int q = 0; q < Q; ++q) {
                    double m = 0.0;
                    for (int a = 0; a < D; ++a) m += (up[a][q] - dn[a][q]) * s[a];
                    const double ftp = 4.0 / 3.0 * w->phi[ce * Q + q] - 1.0 / 3.0 * fin[q * nc + ci];
                    fout[q * nc + ci] = ftp - dt / V * m;
                }
            }
}

int oracle_step(const oracle_cfg* cfg, const double* fin, double* fout, const double* force, double t)
{
    return oracle_run(cfg, fin, fout, force, t, 1);
}

/* nsteps steps from t0 (time t0 + i dt at step i), f_in -> f_out; f_out may
 * equal f_in */
int oracle_run(const oracle_cfg* cfg, const double* fin, double* fout, const double* force, double t0,
               int nsteps)
{
    octx o;
    if (nsteps < 0) return -1;
    if (setup(&o, cfg)) return -1;
    oworkspace w;
    const size_t len = (size_t)ncells(&o) * o.Q;
    double* tmp = (double*)malloc(sizeof(double) * len);
    if (work_alloc(&o, force, &w) || !tmp) {
        work_free(&w);
        free(tmp);
        ctx_free(&o);
        return -1;
    }
    if (fout != fin) memcpy(fout, fin, sizeof(double) * len);
    double t = t0;
    for (int s = 0; s < nsteps; ++s) {
        step_with(&o, cfg, &w, fout, tmp, t);
        memcpy(fout, tmp, sizeof(double) * len);
        t += cfg->dt;
    }
    free(tmp);
    work_free(&w);
    ctx_free(&o);
    return 0;
}

/* f-bar(x_b, t_n + h) on every interface of axis `axis` before the wall
 * rules, from given f-bar-plus values phi[q][cells] at the centres (ghosts
 * by the same rule as in the step): the interface reconstruction of
 * Eq. (gradient) on its own, for tests.  out[q][faces] with the interface
 * layout of axis `axis` ([z][y][x], n+1 along the axis). */
int oracle_interface_values(const oracle_cfg* cfg, int axis, const double* phi_cells, double* out)
{
    octx o;
    if (setup(&o, cfg)) return -1;
    if (axis < 0 || axis >= o.D) { ctx_free(&o); return -1; }
    const int Q = o.Q;
    const long nc = ncells(&o), nf = face_count(&o, axis);
    double* phi = (double*)calloc((size_t)ncells_ext(&o) * Q, sizeof(double));
    for (int k = 0; k < o.n[2]; ++k)
        for (int j = 0; j < o.n[1]; ++j)
            for (int i = 0; i < o.n[0]; ++i)
                for (int q = 0; q < Q; ++q)
                    phi[cell_ext(&o, i, j, k) * Q + q] = phi_cells[q * nc + cell_int(&o, i, j, k)];
    ghost_fill(&o, phi, Q);
    const double h = 0.5 * cfg->dt;
    const int d0 = face_dim(&o, axis, 0), d1 = face_dim(&o, axis, 1), d2 = face_dim(&o, axis, 2);
    for (int k = 0; k < d2; ++k)
        for (int j = 0; j < d1; ++j)
            for (int i = 0; i < d0; ++i) {
                const int c[3] = {i, j, k};
                double fb[MAXQ];
                interface_fbar(&o, phi, axis, c, h, fb);
                for (int q = 0; q < Q; ++q) out[q * nf + face_idx(&o, axis, c)] = fb[q];
            }
    free(phi);
    ctx_free(&o);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* outputs: Eq. (macro_values) at t, p = (rho - rho0) RT (gauge pressure,   */
/* both models)                                                              */
/* ------------------------------------------------------------------------ */
int oracle_moments(const oracle_cfg* cfg, const double* f, const double* force, double t,
                   double* rho, double* u, double* p, double* totals)
{
    octx o;
    if (setup(&o, cfg)) return -1;
    const int D = o.D, Q = o.Q;
    const long nc = ncells(&o);
    const double gt = gtime(cfg, t);
    double tot[6] = {0, 0, 0, 0, 0, 0};
    for (int k = 0; k < o.n[2]; ++k)
        for (int j = 0; j < o.n[1]; ++j)
            for (int i = 0; i < o.n[0]; ++i) {
                int c[3] = {i, j, k};
                long ci = cell_int(&o, i, j, k);
                double r = 0.0, m[3] = {0, 0, 0}, uu[3] = {0, 0, 0};
                for (int q = 0; q < Q; ++q) {
                    double fq = f[q * nc + ci];
                    if (!isfinite(fq)) tot[5] += 1.0;
                    r += fq;
                    for (int a = 0; a < D; ++a) m[a] += o.xi[q][a] * fq;
                }
                double V = 1.0;
                for (int a = 0; a < D; ++a) V *= o.dl[a][c[a]];
                double k2 = 0.0;
                for (int a = 0; a < D; ++a) {
                    double G = gt * (cfg->G[a] + (force ? force[a * nc + ci] : 0.0));
                    const double rm = mom_density(cfg, r);
                    uu[a] = (m[a] + rm * G * cfg->dt / 2.0) / rm;
                    k2 += uu[a] * uu[a];
                    if (u) u[a * nc + ci] = uu[a];
                    tot[1 + a] += V * m[a];
                }
                if (rho) rho[ci] = r;
                if (p) p[ci] = (r - cfg->rho0) * cfg->RT;
                tot[0] += V * r;
                tot[4] += 0.5 * V * k2;
            }
    if (totals)
        for (int m = 0; m < 6; ++m) totals[m] = tot[m];
    ctx_free(&o);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* reverse mode (tape-free: forward intermediates are recomputed)            */
/* ------------------------------------------------------------------------ */

/* partial derivatives of feq_q and S_q with respect to rho, u, G */
static void feq_partials(const octx* o, const oracle_cfg* cfg, int q, double rho, const double* u,
                         const double* G, double* dfe_dr, double* dfe_du, double* dS_dr,
                         double* dS_du, double* dS_dG)
{
    const int D = o->D;
    const double RT = cfg->RT, rho0 = cfg->rho0;
    double xu = 0.0, gx = 0.0;
    for (int a = 0; a < D; ++a) { xu += o->xi[q][a] * u[a]; gx += G[a] * (o->xi[q][a] - u[a]); }
    double fe = feq_q(o, cfg, q, rho, u);
    *dfe_dr = o->W[q];
    *dS_dr = gx / RT * o->W[q];
    for (int a = 0; a < 3; ++a) { dfe_du[a] = 0; dS_du[a] = 0; dS_dG[a] = 0; }
    for (int a = 0; a < D; ++a) {
        dfe_du[a] = o->W[q] * rho0 * (o->xi[q][a] / RT + xu * o->xi[q][a] / (RT * RT) - u[a] / RT);
        dS_du[a] = -G[a] / RT * fe + gx / RT * dfe_du[a];
        dS_dG[a] = (o->xi[q][a] - u[a]) / RT * fe;
    }
}

static inline int wrapi(int i, int n) { return ((i % n) + n) % n; }

/* Eq. (gradient) for one velocity q on the interface of axis a with
 * coordinates c (c[a] = interface index): the same value as interface_fbar,
 * written with the bilinear weights explicit so that face_value_adj below is
 * visibly its transpose. */
static double face_value(const octx* o, const double* fp, int a, const int* c, int q, double h)
{
    const int D = o->D, Q = o->Q;
    int cl[3] = {c[0], c[1], c[2]};
    cl[a] -= 1;
    const double w = o->w[a][c[a]], gn = o->g[a][c[a]];
    const long L = cell_ext(o, cl[0], cl[1], cl[2]), R = cell_ext(o, c[0], c[1], c[2]);
    double sig[3] = {0, 0, 0};
    sig[a] = gn * (fp[R * Q + q] - fp[L * Q + q]);
    for (int b = 0; b < D; ++b) {
        if (b == a) continue;
        double ev[2];
        for (int up = 0; up < 2; ++up) {
            int ce_[3] = {c[0], c[1], c[2]};
            ce_[b] += up;
            const double wa = o->w[a][ce_[a]], wb = o->w[b][ce_[b]];
            int c00[3] = {ce_[0], ce_[1], ce_[2]}, c10[3] = {ce_[0], ce_[1], ce_[2]};
            int c01[3] = {ce_[0], ce_[1], ce_[2]}, c11[3] = {ce_[0], ce_[1], ce_[2]};
            c00[a] -= 1; c00[b] -= 1; c10[b] -= 1; c01[a] -= 1;
            const double e1 = (1.0 - wa) * fp[cell_ext(o, c00[0], c00[1], c00[2]) * Q + q] +
                              wa * fp[cell_ext(o, c10[0], c10[1], c10[2]) * Q + q];
            const double e2 = (1.0 - wa) * fp[cell_ext(o, c01[0], c01[1], c01[2]) * Q + q] +
                              wa * fp[cell_ext(o, c11[0], c11[1], c11[2]) * Q + q];
            ev[up] = (1.0 - wb) * e1 + wb * e2;
        }
        sig[b] = (ev[1] - ev[0]) / o->dl[b][c[b]];
    }
    double xs = 0.0;
    for (int b = 0; b < D; ++b) xs += o->xi[q][b] * sig[b];
    return (1.0 - w) * fp[L * Q + q] + w * fp[R * Q + q] - h * xs;
}

/* transpose of face_value: fpb += Fq * dF/dfp */
static void face_value_adj(const octx* o, double* fpb, int a, const int* c, int q, double h, double Fq)
{
    const int D = o->D, Q = o->Q;
    int cl[3] = {c[0], c[1], c[2]};
    cl[a] -= 1;
    const double w = o->w[a][c[a]], gn = o->g[a][c[a]];
    const long L = cell_ext(o, cl[0], cl[1], cl[2]), R = cell_ext(o, c[0], c[1], c[2]);
    fpb[L * Q + q] += (1.0 - w) * Fq;
    fpb[R * Q + q] += w * Fq;
    const double sa = -h * o->xi[q][a] * Fq;
    fpb[R * Q + q] += gn * sa;
    fpb[L * Q + q] -= gn * sa;
    for (int b = 0; b < D; ++b) {
        if (b == a) continue;
        const double sb = -h * o->xi[q][b] * Fq / o->dl[b][c[b]];
        for (int up = 0; up < 2; ++up) {
            const double sgn = up ? sb : -sb;
            int ce_[3] = {c[0], c[1], c[2]};
            ce_[b] += up;
            const double wa = o->w[a][ce_[a]], wb = o->w[b][ce_[b]];
            int c00[3] = {ce_[0], ce_[1], ce_[2]}, c10[3] = {ce_[0], ce_[1], ce_[2]};
            int c01[3] = {ce_[0], ce_[1], ce_[2]}, c11[3] = {ce_[0], ce_[1], ce_[2]};
            c00[a] -= 1; c00[b] -= 1; c10[b] -= 1; c01[a] -= 1;
            fpb[cell_ext(o, c00[0], c00[1], c00[2]) * Q + q] += (1.0 - wb) * (1.0 - wa) * sgn;
            fpb[cell_ext(o, c10[0], c10[1], c10[2]) * Q + q] += (1.0 - wb) * wa * sgn;
            fpb[cell_ext(o, c01[0], c01[1], c01[2]) * Q + q] += wb * (1.0 - wa) * sgn;
            fpb[cell_ext(o, c11[0], c11[1], c11[2]) * Q + q] += wb * wa * sgn;
        }
    }
}

/* transpose of ghost_fill: fold the adjoint of every ghost point back into
 * the points it was made from, axes in the reverse of the forward order */
static void ghost_fold(const octx* o, double* v, int ncomp)
{
    for (int a = o->D - 1; a >= 0; --a) {
        int lo[3], hi[3];
        for (int b = 0; b < 3; ++b) {
            if (b >= o->D) { lo[b] = 0; hi[b] = 0; continue; }
            if (b < a) { lo[b] = -1; hi[b] = o->n[b]; }
            else { lo[b] = 0; hi[b] = o->n[b] - 1; }
        }
        const int N = o->n[a];
        for (int side = 0; side < 2; ++side) {
            lo[a] = hi[a] = side ? N : -1;
            for (int k = lo[2]; k <= hi[2]; ++k)
                for (int j = lo[1]; j <= hi[1]; ++j)
                    for (int i = lo[0]; i <= hi[0]; ++i) {
                        int c0[3] = {i, j, k}, c1[3] = {i, j, k};
                        const long dst = cell_ext(o, i, j, k);
                        if (o->per[a]) {
                            c0[a] = side ? 0 : N - 1;
                            const long src = cell_ext(o, c0[0], c0[1], c0[2]);
                            for (int m = 0; m < ncomp; ++m) v[src * ncomp + m] += v[dst * ncomp + m];
                        } else {
                            const double r = side ? o->rhi[a] : o->rlo[a];
                            c0[a] = side ? N - 1 : 0;
                            c1[a] = side ? N - 2 : 1;
                            const long s0 = cell_ext(o, c0[0], c0[1], c0[2]);
                            const long s1 = cell_ext(o, c1[0], c1[1], c1[2]);
                            for (int m = 0; m < ncomp; ++m) {
                                v[s0 * ncomp + m] += (1.0 - r) * v[dst * ncomp + m];
                                v[s1 * ncomp + m] += r * v[dst * ncomp + m];
                            }
                        }
                        for (int m = 0; m < ncomp; ++m) v[dst * ncomp + m] = 0.0;
                    }
        }
    }
}

/* interface moments of a set of f-bar values (Eq. (macro_values) with G at
 * the interface and h/2; model 0) */
static void face_macro(const octx* o, const oracle_cfg* cfg, const double* Fb, const double* G, double h,
                       double* rho, double* u)
{
    double r = 0.0, m[3] = {0, 0, 0};
    for (int q = 0; q < o->Q; ++q) {
        r += Fb[q];
        for (int b = 0; b < o->D; ++b) m[b] += o->xi[q][b] * Fb[q];
    }
    *rho = r;
    for (int b = 0; b < 3; ++b) u[b] = 0.0;
    for (int b = 0; b < o->D; ++b) u[b] = (m[b] + cfg->rho0 * G[b] * h / 2.0) / cfg->rho0;
}

/* Reverse mode of one step (incompressible model) on any mesh and boundary
 * set: the forward intermediates are recomputed (no tape), then every step
 * of the forward is transposed in reverse order: the cell update
 * (Eqs. (f_tilde_+), (evolution_equation)), the original distribution at the
 * interfaces (inverse of Eq. (original_f) with the interface moments), the
 * wall rules (Eq. (BB) is a permutation plus a constant; the
 * NEQ rules depend on the moments and values of the opposite interface of
 * the wall cell), the reconstruction (Eq. (gradient)), the ghost layer and
 * Eq. (f_bar_+) with the macroscopic recovery (Eq. (macro_values)).  Face n of a
 * periodic axis is computed by the forward step as a face of its own (equal
 * to face 0), and is transposed as one. */
int oracle_step_adjoint(const oracle_cfg* cfg, const double* fin, const double* force, double t,
                        const double* lam, double* lam_out, double* grad_force)
{
    octx o;
    if (cfg->model != 0) return -2; /* derived for the incompressible model */
    if (setup(&o, cfg)) return -1;
    const int D = o.D, Q = o.Q;
    const long nc = ncells(&o), nce = ncells_ext(&o);
    const double dt = cfg->dt, h = 0.5 * dt, tau = cfg->tau, rho0 = cfg->rho0, RT = cfg->RT;
    const double A1 = (2.0 * tau - h) / (2.0 * tau + dt);
    const double B1 = 3.0 * h / (2.0 * tau + dt);
    const double C1 = 3.0 * tau * h / (2.0 * tau + dt);
    const double A7 = 2.0 * tau / (2.0 * tau + h);
    const double B7 = h / (2.0 * tau + h);
    const double C7 = tau * h / (2.0 * tau + h);
    const double gt = gtime(cfg, t), gth = gtime(cfg, t + h);

    /* ---- forward recomputation: cell transform, ghosts, reconstruction, wall rules ---- */
    double* Gext = force_ext(&o, force);
    double* fp = (double*)calloc((size_t)nce * Q, sizeof(double));
    double* rho_c = (double*)calloc((size_t)nc, sizeof(double));
    double* u_c = (double*)calloc((size_t)nc * 3, sizeof(double));
    double* G_c = (double*)calloc((size_t)nc * 3, sizeof(double));
    for (int k = 0; k < o.n[2]; ++k)
        for (int j = 0; j < o.n[1]; ++j)
            for (int i = 0; i < o.n[0]; ++i) {
                long ci = cell_int(&o, i, j, k), ce = cell_ext(&o, i, j, k);
                double rho = 0.0, m[3] = {0, 0, 0}, G[3], u[3] = {0, 0, 0};
                for (int q = 0; q < Q; ++q) {
                    double fq = fin[q * nc + ci];
                    rho += fq;
                    for (int a = 0; a < D; ++a) m[a] += o.xi[q][a] * fq;
                }
                accel_cell(&o, cfg, Gext, ce, gt, G);
                for (int a = 0; a < D; ++a) u[a] = (m[a] + rho0 * G[a] * dt / 2.0) / rho0;
                rho_c[ci] = rho;
                for (int a = 0; a < 3; ++a) { u_c[ci * 3 + a] = u[a]; G_c[ci * 3 + a] = G[a]; }
                for (int q = 0; q < Q; ++q)
                    fp[ce * Q + q] = A1 * fin[q * nc + ci] + B1 * feq_q(&o, cfg, q, rho, u) +
                                     C1 * src_q(&o, cfg, q, rho, u, G);
            }
    ghost_fill(&o, fp, Q);

    /* F4: f-bar on the interfaces from Eq. (gradient); F5: after the wall rules */
    double* F4[3] = {NULL, NULL, NULL};
    double* F5[3] = {NULL, NULL, NULL};
    double* Fb5[3] = {NULL, NULL, NULL}; /* adjoint of F5, then of F4 */
    double* Gbf[3] = {NULL, NULL, NULL}; /* adjoint of the face acceleration */
    for (int a = 0; a < D; ++a) {
        long nf = face_count(&o, a);
        F4[a] = (double*)malloc(sizeof(double) * nf * Q);
        F5[a] = (double*)malloc(sizeof(double) * nf * Q);
        Fb5[a] = (double*)calloc((size_t)nf * Q, sizeof(double));
        Gbf[a] = (double*)calloc((size_t)nf * 3, sizeof(double));
        int d0 = face_dim(&o, a, 0), d1 = face_dim(&o, a, 1), d2 = face_dim(&o, a, 2);
        for (int k = 0; k < d2; ++k)
            for (int j = 0; j < d1; ++j)
                for (int i = 0; i < d0; ++i) {
                    int c[3] = {i, j, k};
                    long fi = face_idx(&o, a, c);
                    for (int q = 0; q < Q; ++q) {
                        F4[a][fi * Q + q] = face_value(&o, fp, a, c, q, h);
                        F5[a][fi * Q + q] = F4[a][fi * Q + q];
                    }
                }
    }
    for (int s = 0; s < 2 * D; ++s) {
        int a = s / 2, hi = s % 2;
        if (o.per[a]) continue;
        int bc = cfg->bc[s], N = o.n[a];
        int nsg = hi ? 1 : -1;
        int lo[3] = {0, 0, 0}, up[3];
        for (int b = 0; b < 3; ++b) up[b] = o.n[b] - 1;
        lo[a] = up[a] = 0;
        for (int k = lo[2]; k <= up[2]; ++k)
            for (int j = lo[1]; j <= up[1]; ++j)
                for (int i = lo[0]; i <= up[0]; ++i) {
                    int cw[3] = {i, j, k}, co[3] = {i, j, k};
                    cw[a] = hi ? N : 0;
                    co[a] = hi ? N - 1 : 1;
                    const double* Pw = F4[a] + face_idx(&o, a, cw) * Q;
                    double* Fw = F5[a] + face_idx(&o, a, cw) * Q;
                    const double* Fo = F4[a] + face_idx(&o, a, co) * Q;
                    if (bc == OR_BOUNCE_BACK) {
                        for (int q = 0; q < Q; ++q) {
                            if (o.e[q][a] * nsg >= 0) continue;
                            double xu = 0.0;
                            for (int b = 0; b < D; ++b) xu += o.xi[q][b] * cfg->uw[s][b];
                            Fw[q] = Pw[o.opp[q]] + 2.0 * rho0 * o.W[q] * xu / RT;
                        }
                    } else {
                        double rc, uc[3], Gb[3], ra, ua[3] = {0, 0, 0};
                        accel_face(&o, cfg, Gext, a, co, gth, Gb);
                        face_macro(&o, cfg, Fo, Gb, h, &rc, uc);
                        if (bc == OR_NEQ_VELOCITY) {
                            ra = rc;
                            for (int b = 0; b < D; ++b) ua[b] = cfg->uw[s][b];
                        } else {
                            ra = pressure_wall_density(cfg, s, gth);
                            for (int b = 0; b < D; ++b) ua[b] = uc[b];
                        }
                        for (int q = 0; q < Q; ++q) {
                            if (o.e[q][a] * nsg >= 0) continue;
                            Fw[q] = feq_q(&o, cfg, q, ra, ua) + (Fo[q] - feq_q(&o, cfg, q, rc, uc));
                        }
                    }
                }
    }

    /* ---- reverse sweep ---- */
    double* fpb = (double*)calloc((size_t)nce * Q, sizeof(double));  /* adjoint of f-bar-plus (ext) */
    double* Gb_sp = (double*)calloc((size_t)nce * 3, sizeof(double)); /* adjoint of the spatial force (ext) */
    for (long c = 0; c < nc * Q; ++c) lam_out[c] = 0.0;

    /* Eqs. (f_tilde_+), (evolution_equation): f~new = 4/3 f-bar-plus - 1/3 f~ - dt/V sum_faces (xi.n) f s */
    for (int k = 0; k < o.n[2]; ++k)
        for (int j = 0; j < o.n[1]; ++j)
            for (int i = 0; i < o.n[0]; ++i) {
                long ci = cell_int(&o, i, j, k), ce = cell_ext(&o, i, j, k);
                for (int q = 0; q < Q; ++q) {
                    fpb[ce * Q + q] += 4.0 / 3.0 * lam[q * nc + ci];
                    lam_out[q * nc + ci] += -1.0 / 3.0 * lam[q * nc + ci];
                }
            }

    /* inverse of Eq. (original_f) at every interface, from the flux adjoint of its (at most two) cells */
    for (int a = 0; a < D; ++a) {
        int d0 = face_dim(&o, a, 0), d1 = face_dim(&o, a, 1), d2 = face_dim(&o, a, 2);
        int N = o.n[a];
        for (int k = 0; k < d2; ++k)
            for (int j = 0; j < d1; ++j)
                for (int i = 0; i < d0; ++i) {
                    int c[3] = {i, j, k};
                    long fi = face_idx(&o, a, c);
                    double Fo_b[MAXQ];
                    for (int q = 0; q < Q; ++q) Fo_b[q] = 0.0;
                    for (int side = 0; side < 2; ++side) {
                        int cc[3] = {i, j, k};
                        cc[a] = side ? c[a] : c[a] - 1; /* side 0: the cell below (this is its + face) */
                        if (cc[a] < 0 || cc[a] >= N) continue;
                        double V = 1.0, sf = 1.0;
                        for (int b = 0; b < D; ++b) {
                            V *= o.dl[b][cc[b]];
                            if (b != a) sf *= o.dl[b][cc[b]];
                        }
                        long cidx = cell_int(&o, cc[0], cc[1], cc[2]);
                        double sgn = side ? 1.0 : -1.0;
                        for (int q = 0; q < Q; ++q) Fo_b[q] += sgn * dt / V * o.xi[q][a] * sf * lam[q * nc + cidx];
                    }
                    const double* Fb = F5[a] + fi * Q;
                    double rho, u[3], G[3];
                    accel_face(&o, cfg, Gext, a, c, gth, G);
                    face_macro(&o, cfg, Fb, G, h, &rho, u);
                    double rb = 0.0, ub[3] = {0, 0, 0}, Gbb[3] = {0, 0, 0};
                    for (int q = 0; q < Q; ++q) {
                        double dfr, dfu[3], dsr, dsu[3], dsg[3];
                        feq_partials(&o, cfg, q, rho, u, G, &dfr, dfu, &dsr, dsu, dsg);
                        Fb5[a][fi * Q + q] = A7 * Fo_b[q];
                        rb += Fo_b[q] * (B7 * dfr + C7 * dsr);
                        for (int b = 0; b < D; ++b) {
                            ub[b] += Fo_b[q] * (B7 * dfu[b] + C7 * dsu[b]);
                            Gbb[b] += Fo_b[q] * C7 * dsg[b];
                        }
                    }
                    for (int b = 0; b < D; ++b) Gbb[b] += ub[b] * h / 2.0;
                    for (int q = 0; q < Q; ++q) {
                        double v = rb;
                        for (int b = 0; b < D; ++b) v += o.xi[q][b] * ub[b] / rho0;
                        Fb5[a][fi * Q + q] += v;
                    }
                    for (int b = 0; b < D; ++b) Gbf[a][fi * 3 + b] += Gbb[b];
                }
    }

    /* wall rules transposed: Fb5 of wall faces becomes the adjoint of F4; NEQ
     * adds to the opposite interface of the wall cell */
    for (int s = 0; s < 2 * D; ++s) {
        int a = s / 2, hi = s % 2;
        if (o.per[a]) continue;
        int bc = cfg->bc[s], N = o.n[a];
        int nsg = hi ? 1 : -1;
        int lo[3] = {0, 0, 0}, up[3];
        for (int b = 0; b < 3; ++b) up[b] = o.n[b] - 1;
        lo[a] = up[a] = 0;
        for (int k = lo[2]; k <= up[2]; ++k)
            for (int j = lo[1]; j <= up[1]; ++j)
                for (int i = lo[0]; i <= up[0]; ++i) {
                    int cw[3] = {i, j, k}, co[3] = {i, j, k};
                    cw[a] = hi ? N : 0;
                    co[a] = hi ? N - 1 : 1;
                    double* Bw = Fb5[a] + face_idx(&o, a, cw) * Q;
                    double* Bo = Fb5[a] + face_idx(&o, a, co) * Q;
                    double rep[MAXQ];
                    for (int q = 0; q < Q; ++q) {
                        rep[q] = (o.e[q][a] * nsg < 0) ? Bw[q] : 0.0;
                        if (o.e[q][a] * nsg < 0) Bw[q] = 0.0;
                    }
                    if (bc == OR_BOUNCE_BACK) {
                        for (int q = 0; q < Q; ++q)
                            if (o.e[q][a] * nsg < 0) Bw[o.opp[q]] += rep[q];
                    } else {
                        const double* Fo = F4[a] + face_idx(&o, a, co) * Q;
                        double rc, uc[3], Gb[3], ra, ua[3] = {0, 0, 0};
                        accel_face(&o, cfg, Gext, a, co, gth, Gb);
                        face_macro(&o, cfg, Fo, Gb, h, &rc, uc);
                        const int vel = (bc == OR_NEQ_VELOCITY);
                        if (vel) {
                            ra = rc;
                            for (int b = 0; b < D; ++b) ua[b] = cfg->uw[s][b];
                        } else {
                            ra = pressure_wall_density(cfg, s, gth);
                            for (int b = 0; b < D; ++b) ua[b] = uc[b];
                        }
                        double rcb = 0.0, ucb[3] = {0, 0, 0};
                        for (int q = 0; q < Q; ++q) {
                            if (o.e[q][a] * nsg >= 0) continue;
                            double dfr, dfu[3], dsr, dsu[3], dsg[3];
                            /* + feq(ra, ua) */
                            feq_partials(&o, cfg, q, ra, ua, Gb, &dfr, dfu, &dsr, dsu, dsg);
                            if (vel) rcb += rep[q] * dfr;
                            else
                                for (int b = 0; b < D; ++b) ucb[b] += rep[q] * dfu[b];
                            /* + Fo - feq(rc, uc) */
                            Bo[q] += rep[q];
                            feq_partials(&o, cfg, q, rc, uc, Gb, &dfr, dfu, &dsr, dsu, dsg);
                            rcb -= rep[q] * dfr;
                            for (int b = 0; b < D; ++b) ucb[b] -= rep[q] * dfu[b];
                        }
                        for (int q = 0; q < Q; ++q) {
                            double v = rcb;
                            for (int b = 0; b < D; ++b) v += o.xi[q][b] * ucb[b] / rho0;
                            Bo[q] += v;
                        }
                        for (int b = 0; b < D; ++b) Gbf[a][face_idx(&o, a, co) * 3 + b] += ucb[b] * h / 2.0;
                    }
                }
    }

    /* Eq. (gradient) transposed, and the face acceleration (interpolated like
     * f-bar-plus along the normal, at t_n + h) */
    for (int a = 0; a < D; ++a) {
        int d0 = face_dim(&o, a, 0), d1 = face_dim(&o, a, 1), d2 = face_dim(&o, a, 2);
        for (int k = 0; k < d2; ++k)
            for (int j = 0; j < d1; ++j)
                for (int i = 0; i < d0; ++i) {
                    int c[3] = {i, j, k}, cl[3] = {i, j, k};
                    cl[a] -= 1;
                    long fi = face_idx(&o, a, c);
                    for (int q = 0; q < Q; ++q) face_value_adj(&o, fpb, a, c, q, h, Fb5[a][fi * Q + q]);
                    double w = o.w[a][c[a]];
                    long Le = cell_ext(&o, cl[0], cl[1], cl[2]), Re = cell_ext(&o, c[0], c[1], c[2]);
                    for (int b = 0; b < D; ++b) {
                        Gb_sp[Le * 3 + b] += (1.0 - w) * gth * Gbf[a][fi * 3 + b];
                        Gb_sp[Re * 3 + b] += w * gth * Gbf[a][fi * 3 + b];
                    }
                }
    }

    /* ghost layer transposed (f-bar-plus and the spatial force share the rule;
     * the force adjoint is kept with 3 components per point) */
    ghost_fold(&o, fpb, Q);
    {
        double* g = (double*)calloc((size_t)nce * D, sizeof(double));
        for (long e = 0; e < nce; ++e)
            for (int b = 0; b < D; ++b) g[e * D + b] = Gb_sp[e * 3 + b];
        ghost_fold(&o, g, D);
        for (long e = 0; e < nce; ++e)
            for (int b = 0; b < 3; ++b) Gb_sp[e * 3 + b] = b < D ? g[e * D + b] : 0.0;
        free(g);
    }

    /* Eq. (f_bar_+) with Eq. (macro_values) transposed */
    for (int k = 0; k < o.n[2]; ++k)
        for (int j = 0; j < o.n[1]; ++j)
            for (int i = 0; i < o.n[0]; ++i) {
                long ci = cell_int(&o, i, j, k), ce = cell_ext(&o, i, j, k);
                double rho = rho_c[ci], u[3], G[3];
                for (int a = 0; a < 3; ++a) { u[a] = u_c[ci * 3 + a]; G[a] = G_c[ci * 3 + a]; }
                double rb = 0.0, ub[3] = {0, 0, 0}, Gcb[3] = {0, 0, 0};
                for (int q = 0; q < Q; ++q) {
                    double pb = fpb[ce * Q + q];
                    double dfr, dfu[3], dsr, dsu[3], dsg[3];
                    feq_partials(&o, cfg, q, rho, u, G, &dfr, dfu, &dsr, dsu, dsg);
                    lam_out[q * nc + ci] += A1 * pb;
                    rb += pb * (B1 * dfr + C1 * dsr);
                    for (int b = 0; b < D; ++b) {
                        ub[b] += pb * (B1 * dfu[b] + C1 * dsu[b]);
                        Gcb[b] += pb * C1 * dsg[b];
                    }
                }
                double mb[3] = {0, 0, 0};
                for (int b = 0; b < D; ++b) { mb[b] = ub[b] / rho0; Gcb[b] += ub[b] * dt / 2.0; }
                for (int q = 0; q < Q; ++q) {
                    double v = rb;
                    for (int b = 0; b < D; ++b) v += o.xi[q][b] * mb[b];
                    lam_out[q * nc + ci] += v;
                }
                if (grad_force)
                    for (int b = 0; b < D; ++b)
                        grad_force[b * nc + ci] += gt * Gcb[b] + Gb_sp[ce * 3 + b];
            }

    for (int a = 0; a < 3; ++a) { free(F4[a]); free(F5[a]); free(Fb5[a]); free(Gbf[a]); }
    free(fp); free(fpb); free(Gb_sp); free(rho_c); free(u_c); free(G_c); free(Gext);
    ctx_free(&o);
    return 0;
}

int oracle_init_adjoint(const oracle_cfg* cfg, const double* u, const double* force, double t0,
                        const double* lam0, double* grad_u, double* grad_force)
{
    octx o;
    if (cfg->model != 0) return -2; /* derived for the incompressible model */
    if (setup(&o, cfg)) return -1;
    const int D = o.D, Q = o.Q;
    const long nc = ncells(&o);
    const double gt = gtime(cfg, t0), rho = cfg->rho0;
    for (long c = 0; c < nc; ++c) {
        double uu[3] = {0, 0, 0}, G[3] = {0, 0, 0};
        for (int a = 0; a < D; ++a) {
            if (u) uu[a] = u[a * nc + c];
            G[a] = gt * (cfg->G[a] + (force ? force[a * nc + c] : 0.0));
        }
        double gu[3] = {0, 0, 0}, gG[3] = {0, 0, 0};
        for (int q = 0; q < Q; ++q) {
            double dfr, dfu[3], dsr, dsu[3], dsg[3];
            feq_partials(&o, cfg, q, rho, uu, G, &dfr, dfu, &dsr, dsu, dsg);
            double l = lam0[q * nc + c];
            for (int a = 0; a < D; ++a) {
                gu[a] += l * (dfu[a] - 0.5 * cfg->dt * dsu[a]);
                gG[a] += l * (-0.5 * cfg->dt * dsg[a]);
            }
        }
        for (int a = 0; a < D; ++a) {
            if (grad_u) grad_u[a * nc + c] += gu[a];
            if (grad_force) grad_force[a * nc + c] += gt * gG[a];
        }
    }
    ctx_free(&o);
    return 0;
}
