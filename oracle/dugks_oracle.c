/*
 * dugks_oracle.c -- plain FP64 CPU oracle of one incompressible-DUGKS step
 * with body force (arXiv:1411.6121).
 *
 * TEST INFRASTRUCTURE ONLY: used by the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg.  It is deliberately slow and literal:
 * every stage of the Appendix algorithm writes its own array over its own
 * point set (X_c, X_cg, X_b, X_bc), in the order the Appendix gives, with no
 * blocking or fusion.  It shares no code with the HIP path.
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

/* face coordinates of one axis: uniform, or the tanh stretching of
 * Eq. (Nonuniform_mesh): zeta_i = 1/2 + tanh(k(i/N - 1/2)) / (2 tanh(k/2)) */
static void make_faces(int kind, int N, double L, double k, double* X)
{
    for (int i = 0; i <= N; ++i) {
        if (kind == OR_TANH) {
            double zeta = 0.5 + tanh(k * ((double)i / N - 0.5)) / (2.0 * tanh(0.5 * k));
            X[i] = L * zeta;
        } else {
            X[i] = L * (double)i / N;
        }
    }
    X[0] = 0.0;
    X[N] = L;
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
        make_faces(cfg->mesh[a], N, L, cfg->k_stretch, o->X[a]);
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

/* Eq. (S), evaluated with the incompressible equilibrium as the Appendix
 * does: S = G.(xi - u)/RT feq */
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

/* Step 2 (ghost points X_cg), for any field with ncomp values per point.
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
 * the spatial part is interpolated like f-bar-plus (step 3) */
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
/* the step (Appendix, steps 1-9; step 10 is oracle_moments)                 */
/* ------------------------------------------------------------------------ */
int oracle_step(const oracle_cfg* cfg, const double* fin, double* fout, const double* force,
                double t)
{
    octx o;
    if (setup(&o, cfg)) return -1;
    const int D = o.D, Q = o.Q;
    const long nc = ncells(&o), nce = ncells_ext(&o);
    const double dt = cfg->dt, h = 0.5 * dt, tau = cfg->tau, rho0 = cfg->rho0, RT = cfg->RT;
    /* Eq. (f_bar_+) */
    const double A1 = (2.0 * tau - h) / (2.0 * tau + dt);
    const double B1 = 3.0 * h / (2.0 * tau + dt);
    const double C1 = 3.0 * tau * h / (2.0 * tau + dt);
    /* step 7, inverse of Eq. (original_f) */
    const double A7 = 2.0 * tau / (2.0 * tau + h);
    const double B7 = h / (2.0 * tau + h);
    const double C7 = tau * h / (2.0 * tau + h);
    const double gt = gtime(cfg, t), gth = gtime(cfg, t + h);

    double* Gext = force_ext(&o, force);
    double* fp = (double*)calloc((size_t)nce * Q, sizeof(double)); /* f-bar-plus on X_c u X_cg */
    double* F[3] = {NULL, NULL, NULL};                             /* values on X_b           */
    double* Eg[3] = {NULL, NULL, NULL};                            /* f-bar-plus on X_bc      */

    /* Step 1: f-bar-plus at the centres, Eq. (f_bar_+), with rho, u from
     * Eq. (macro_values) at t_n and G(x_c, t_n). */
#pragma omp parallel for collapse(2) schedule(static)
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
                const double rm = mom_density(cfg, rho);
                for (int a = 0; a < D; ++a) u[a] = (m[a] + rm * G[a] * dt / 2.0) / rm;
                for (int q = 0; q < Q; ++q)
                    fp[ce * Q + q] = A1 * fin[q * nc + ci] + B1 * feq_q(&o, cfg, q, rho, u) +
                                     C1 * src_q(&o, cfg, q, rho, u, G);
            }

    /* Step 2: ghost points */
    ghost_fill(&o, fp, Q);

    /* Step 3: f-bar-plus at X_b (face mid-points) and X_bc (cross points) by
     * centre interpolation: linear along the face normal, bilinear in the
     * plane of the two interfaces that cross. */
    for (int a = 0; a < D; ++a) {
        long nf = face_count(&o, a);
        F[a] = (double*)malloc(sizeof(double) * nf * Q);
        int d0 = face_dim(&o, a, 0), d1 = face_dim(&o, a, 1), d2 = face_dim(&o, a, 2);
#pragma omp parallel for collapse(2) schedule(static)
        for (int k = 0; k < d2; ++k)
            for (int j = 0; j < d1; ++j)
                for (int i = 0; i < d0; ++i) {
                    int c[3] = {i, j, k}, cl[3] = {i, j, k};
                    cl[a] -= 1;
                    double w = o.w[a][c[a]];
                    long L = cell_ext(&o, cl[0], cl[1], cl[2]), R = cell_ext(&o, c[0], c[1], c[2]);
                    long fi = face_idx(&o, a, c);
                    for (int q = 0; q < Q; ++q)
                        F[a][fi * Q + q] = (1.0 - w) * fp[L * Q + q] + w * fp[R * Q + q];
                }
    }
    for (int a = 0; a < D; ++a)
        for (int b = a + 1; b < D; ++b) {
            int p = pair_id(a, b);
            long ne = edge_count(&o, a, b);
            Eg[p] = (double*)malloc(sizeof(double) * ne * Q);
            int d0 = edge_dim(&o, a, b, 0), d1 = edge_dim(&o, a, b, 1), d2 = edge_dim(&o, a, b, 2);
#pragma omp parallel for collapse(2) schedule(static)
            for (int k = 0; k < d2; ++k)
                for (int j = 0; j < d1; ++j)
                    for (int i = 0; i < d0; ++i) {
                        int c[3] = {i, j, k};
                        double wa = o.w[a][c[a]], wb = o.w[b][c[b]];
                        int c00[3] = {i, j, k}, c10[3] = {i, j, k}, c01[3] = {i, j, k}, c11[3] = {i, j, k};
                        c00[a] -= 1; c00[b] -= 1;
                        c10[b] -= 1;
                        c01[a] -= 1;
                        long p00 = cell_ext(&o, c00[0], c00[1], c00[2]);
                        long p10 = cell_ext(&o, c10[0], c10[1], c10[2]);
                        long p01 = cell_ext(&o, c01[0], c01[1], c01[2]);
                        long p11 = cell_ext(&o, c11[0], c11[1], c11[2]);
                        long ei = edge_idx(&o, a, b, c);
                        for (int q = 0; q < Q; ++q) {
                            double e1 = (1.0 - wa) * fp[p00 * Q + q] + wa * fp[p10 * Q + q];
                            double e2 = (1.0 - wa) * fp[p01 * Q + q] + wa * fp[p11 * Q + q];
                            Eg[p][ei * Q + q] = (1.0 - wb) * e1 + wb * e2;
                        }
                    }
        }

    /* Step 4: gradient sigma_b by differences and
     * F(x_b) = f-bar-plus(x_b) - xi h . sigma_b, Eq. (gradient).
     * Normal component: difference of the two centres; tangential
     * components: difference of the two cross points over the face width. */
    for (int a = 0; a < D; ++a) {
        int d0 = face_dim(&o, a, 0), d1 = face_dim(&o, a, 1), d2 = face_dim(&o, a, 2);
#pragma omp parallel for collapse(2) schedule(static)
        for (int k = 0; k < d2; ++k)
            for (int j = 0; j < d1; ++j)
                for (int i = 0; i < d0; ++i) {
                    int c[3] = {i, j, k}, cl[3] = {i, j, k};
                    cl[a] -= 1;
                    long L = cell_ext(&o, cl[0], cl[1], cl[2]), R = cell_ext(&o, c[0], c[1], c[2]);
                    long fi = face_idx(&o, a, c);
                    double gn = o.g[a][c[a]];
                    long e_lo[3] = {0, 0, 0}, e_hi[3] = {0, 0, 0};
                    double inv[3] = {0, 0, 0};
                    for (int b = 0; b < D; ++b) {
                        if (b == a) continue;
                        int cu[3] = {i, j, k}, cd[3] = {i, j, k};
                        cu[b] += 1;
                        e_lo[b] = edge_idx(&o, a, b, cd);
                        e_hi[b] = edge_idx(&o, a, b, cu);
                        inv[b] = 1.0 / o.dl[b][c[b]];
                    }
                    for (int q = 0; q < Q; ++q) {
                        double sig[3] = {0, 0, 0};
                        sig[a] = gn * (fp[R * Q + q] - fp[L * Q + q]);
                        for (int b = 0; b < D; ++b) {
                            if (b == a) continue;
                            const double* Ep = Eg[pair_id(a, b)];
                            sig[b] = (Ep[e_hi[b] * Q + q] - Ep[e_lo[b] * Q + q]) * inv[b];
                        }
                        double xs = 0.0;
                        for (int b = 0; b < D; ++b) xs += o.xi[q][b] * sig[b];
                        F[a][fi * Q + q] = F[a][fi * Q + q] - h * xs;
                    }
                }
    }

    /* Step 5: boundary processing at wall faces, for the velocities leaving
     * the wall into the domain (xi . n < 0, n the outward normal):
     * bounce-back, Eq. (BB), with rho_w = rho0; or non-equilibrium
     * extrapolation, Eq. (NEQ), whose non-equilibrium part is taken at x_c,
     * the opposite interface of the same wall cell, with rho_c, u_c its
     * step-6 moments.  Velocity condition: (rho_c, u_w); pressure
     * condition: (rho0 + p_w/RT, u_c). */
    for (int s = 0; s < 2 * D; ++s) {
        int a = s / 2, hi = s % 2;
        if (o.per[a]) continue;
        int bc = cfg->bc[s];
        int N = o.n[a];
        int fw = hi ? N : 0, fo = hi ? N - 1 : 1;
        int nsg = hi ? 1 : -1;
        int lo[3] = {0, 0, 0}, up[3];
        for (int b = 0; b < 3; ++b) up[b] = o.n[b] - 1;
        lo[a] = up[a] = 0;
#pragma omp parallel for collapse(2) schedule(static)
        for (int k = lo[2]; k <= up[2]; ++k)
            for (int j = lo[1]; j <= up[1]; ++j)
                for (int i = lo[0]; i <= up[0]; ++i) {
                    int cw[3] = {i, j, k}, co[3] = {i, j, k};
                    cw[a] = fw; co[a] = fo;
                    double* Fw = F[a] + face_idx(&o, a, cw) * Q;
                    const double* Fo = F[a] + face_idx(&o, a, co) * Q;
                    double pre[MAXQ];
                    for (int q = 0; q < Q; ++q) pre[q] = Fw[q];
                    if (bc == OR_BOUNCE_BACK) {
                        for (int q = 0; q < Q; ++q) {
                            if (o.e[q][a] * nsg >= 0) continue;
                            double xu = 0.0;
                            for (int b = 0; b < D; ++b) xu += o.xi[q][b] * cfg->uw[s][b];
                            Fw[q] = pre[o.opp[q]] + 2.0 * rho0 * o.W[q] * xu / RT;
                        }
                    } else {
                        double rc = 0.0, m[3] = {0, 0, 0}, Gb[3], uc[3] = {0, 0, 0};
                        for (int q = 0; q < Q; ++q) {
                            rc += Fo[q];
                            for (int b = 0; b < D; ++b) m[b] += o.xi[q][b] * Fo[q];
                        }
                        accel_face(&o, cfg, Gext, a, co, gth, Gb);
                        const double rm = mom_density(cfg, rc);
                        for (int b = 0; b < D; ++b) uc[b] = (m[b] + rm * Gb[b] * h / 2.0) / rm;
                        double ra, ua[3] = {0, 0, 0};
                        if (bc == OR_NEQ_VELOCITY) {
                            ra = rc;
                            for (int b = 0; b < D; ++b) ua[b] = cfg->uw[s][b];
                        } else {
                            ra = rho0 + cfg->pw[s] / RT;
                            for (int b = 0; b < D; ++b) ua[b] = uc[b];
                        }
                        for (int q = 0; q < Q; ++q) {
                            if (o.e[q][a] * nsg >= 0) continue;
                            Fw[q] = feq_q(&o, cfg, q, ra, ua) + (Fo[q] - feq_q(&o, cfg, q, rc, uc));
                        }
                    }
                }
    }

    /* Steps 6-7: interface moments (with + rho0 G h/2) and the original
     * distribution f(x_b, t_n + h), inverse of Eq. (original_f). */
    for (int a = 0; a < D; ++a) {
        int d0 = face_dim(&o, a, 0), d1 = face_dim(&o, a, 1), d2 = face_dim(&o, a, 2);
#pragma omp parallel for collapse(2) schedule(static)
        for (int k = 0; k < d2; ++k)
            for (int j = 0; j < d1; ++j)
                for (int i = 0; i < d0; ++i) {
                    int c[3] = {i, j, k};
                    double* Fb = F[a] + face_idx(&o, a, c) * Q;
                    double rho = 0.0, m[3] = {0, 0, 0}, G[3], u[3] = {0, 0, 0};
                    for (int q = 0; q < Q; ++q) {
                        rho += Fb[q];
                        for (int b = 0; b < D; ++b) m[b] += o.xi[q][b] * Fb[q];
                    }
                    accel_face(&o, cfg, Gext, a, c, gth, G);
                    const double rm = mom_density(cfg, rho);
                    for (int b = 0; b < D; ++b) u[b] = (m[b] + rm * G[b] * h / 2.0) / rm;
                    for (int q = 0; q < Q; ++q)
                        Fb[q] = A7 * Fb[q] + B7 * feq_q(&o, cfg, q, rho, u) + C7 * src_q(&o, cfg, q, rho, u, G);
                }
    }

    /* Steps 8-9: micro-flux m = sum over the cell's faces of (xi.n_j) F s_j,
     * Eq. (microflux) at t_n + h, then f~+ = 4/3 f-bar-plus - 1/3 f~
     * (Eq. (f_tilde_+)) and f~(t+dt) = f~+ - dt/|V| m (Eq. (evolution_equation)). */
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < o.n[2]; ++k)
        for (int j = 0; j < o.n[1]; ++j)
            for (int i = 0; i < o.n[0]; ++i) {
                int c[3] = {i, j, k};
                long ci = cell_int(&o, i, j, k), ce = cell_ext(&o, i, j, k);
                double V = 1.0, s[3] = {1, 1, 1};
                for (int a = 0; a < D; ++a) V *= o.dl[a][c[a]];
                for (int a = 0; a < D; ++a)
                    for (int b = 0; b < D; ++b)
                        if (b != a) s[a] *= o.dl[b][c[b]];
                long fpl[3], fmi[3];
                for (int a = 0; a < D; ++a) {
                    int cp[3] = {i, j, k};
                    cp[a] += 1;
                    fmi[a] = face_idx(&o, a, c);
                    fpl[a] = face_idx(&o, a, cp);
                }
                for (int q = 0; q < Q; ++q) {
                    double m = 0.0;
                    for (int a = 0; a < D; ++a) {
                        m += o.xi[q][a] * F[a][fpl[a] * Q + q] * s[a];   /* n = +e_a */
                        m += -o.xi[q][a] * F[a][fmi[a] * Q + q] * s[a];  /* n = -e_a */
                    }
                    double ftp = 4.0 / 3.0 * fp[ce * Q + q] - 1.0 / 3.0 * fin[q * nc + ci];
                    fout[q * nc + ci] = ftp - dt / V * m;
                }
            }

    for (int a = 0; a < 3; ++a) { free(F[a]); free(Eg[a]); }
    free(fp);
    free(Gext);
    ctx_free(&o);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* step 10 / outputs: Eq. (macro_values), p = (rho - rho0) RT (gauge        */
/* pressure, both models)                                                    */
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

/* Step 3 (cross points) and step 4 for one face value: F(x_b) for velocity
 * q on the face of axis a with coordinates c (c[a] = face index), written
 * out as in the forward step; the reverse scatter below is its transpose. */
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

/* moments of a face value set at time factor gth (steps 6, model 0) */
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
 * of the forward is transposed in reverse order: the update (steps 8-9),
 * the original distribution at the faces (step 7 with the step-6 moments),
 * the wall rules (step 5: bounce-back is a permutation plus a constant; the
 * NEQ rules depend on the moments and values of the opposite interface of
 * the wall cell), the reconstruction (steps 3-4), the ghost points (step 2)
 * and Eq. (f_bar_+) with the macroscopic recovery (step 1).  Face n of a
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

    /* ---- forward recomputation: step 1, step 2, steps 3-4, step 5 ---- */
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

    /* F4: face values after step 4; F5: after the wall rules of step 5 */
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
                            ra = rho0 + cfg->pw[s] / RT;
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

    /* steps 8-9: f~new = 4/3 f-bar-plus - 1/3 f~ - dt/V sum_faces (xi.n) F s */
    for (int k = 0; k < o.n[2]; ++k)
        for (int j = 0; j < o.n[1]; ++j)
            for (int i = 0; i < o.n[0]; ++i) {
                long ci = cell_int(&o, i, j, k), ce = cell_ext(&o, i, j, k);
                for (int q = 0; q < Q; ++q) {
                    fpb[ce * Q + q] += 4.0 / 3.0 * lam[q * nc + ci];
                    lam_out[q * nc + ci] += -1.0 / 3.0 * lam[q * nc + ci];
                }
            }

    /* step 7 at every face, from the flux adjoint of its (at most two) cells */
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

    /* step 5 transposed: Fb5 of wall faces becomes the adjoint of F4; NEQ
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
                            ra = rho0 + cfg->pw[s] / RT;
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

    /* steps 3-4 transposed, and the face acceleration (interpolated like
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

    /* step 2 transposed (f-bar-plus and the spatial force share the rule;
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

    /* step 1 transposed */
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
