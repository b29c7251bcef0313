/*
 * dugks_oracle.h -- plain, slow FP64 CPU oracle of the incompressible DUGKS
 * step with body force (Wu, Shi, Chai & Wang, arXiv:1411.6121).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this code; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no source, header, table
 * or helper with the HIP implementation.
 *
 * The step is written from the equations of Sec. II: a transform of every
 * cell centre (Eqs. (macro_values), (f_bar_+)) with a ghost layer on wall
 * axes, one flux evaluation per interface (Eq. (gradient) with cross-point
 * values for the tangential differences, Eqs. (BB)/(NEQ) on walls, the
 * interface moments, the inverse of Eq. (original_f), Eq. (microflux)), and
 * the conservative cell update (Eqs. (f_tilde_+), (evolution_equation)).
 * Where the paper is silent or garbled, the reading taken is stated at the
 * code that applies it.
 *
 * Array layout at the interface (same as the product's, documented there):
 *   distributions  f[q][z][y][x]  (x fastest), q in the lattice order below
 *   vector fields  v[d][z][y][x]
 *   scalar fields  s[z][y][x]
 */
#ifndef DUGKS_ORACLE_H
#define DUGKS_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_PERIODIC = 0, OR_NEQ_VELOCITY = 1, OR_NEQ_PRESSURE = 2, OR_BOUNCE_BACK = 3 };
enum { OR_UNIFORM = 0, OR_TANH = 1, OR_CUSTOM = 2 };

typedef struct {
    int lattice;        /* 9 (D2Q9), 19 (D3Q19) or 27 (D3Q27) */
    int n[3];           /* cells per axis, n[2] == 1 for D2Q9 */
    double L[3];        /* domain length per axis */
    int mesh[3];        /* OR_UNIFORM, OR_TANH or OR_CUSTOM per axis */
    double k_stretch;   /* tanh stretch constant k */
    double rho0, RT, tau, dt;
    double G[3];        /* uniform part of the acceleration */
    double omega, phase;/* time factor g(t) = cos(omega t + phase) */
    int bc[6];          /* sides -x,+x,-y,+y,-z,+z */
    double uw[6][3];    /* wall velocity per side (velocity BCs) */
    double pw[6];       /* wall pressure per side (pressure BC) */
    int model;          /* 0: incompressible model, Eq. (icfeq) with
                           Eq. (macro_values); 1: original DUGKS, Eq. (feq)
                           with rho u = sum xi f + rho G dt/2 */
    const double* faces[3]; /* OR_CUSTOM axes: the n+1 face coordinates,
                               0 = X_0 < ... < X_n = L */
    double pw_osc[6];   /* oscillating part of the wall pressure: the
                           pressure side holds pw + pw_osc g(t) */
} oracle_cfg;

/* lattice table: e[q*3+a] in {-1,0,1}, w[q]; returns Q or -1 */
int oracle_lattice(int lattice, int* e, double* w);

/* mesh of one axis: faces[n+1], centres[n+2] (ghost, 0..n-1, ghost) */
int oracle_mesh(const oracle_cfg* cfg, int axis, double* faces, double* centres);

/* discrete incompressible equilibrium and force term at one point (all q) */
int oracle_feq(const oracle_cfg* cfg, double rho, const double* u, double* feq);
int oracle_force_term(const oracle_cfg* cfg, double rho, const double* u,
                      const double* G, double* S);

/* f~0 = feq(rho,u) - dt/2 S(rho,u,G(x,t0)); rho, u, force nullable */
int oracle_init(const oracle_cfg* cfg, const double* rho, const double* u,
                const double* force, double t0, double* f_out);

/* one step t_n -> t_n + dt; force nullable (spatial part G^(x), [D][cells]) */
int oracle_step(const oracle_cfg* cfg, const double* f_in, double* f_out,
                const double* force, double t_n);

/* nsteps steps from t0 (step i at t0 + i dt); f_out may equal f_in */
int oracle_run(const oracle_cfg* cfg, const double* f_in, double* f_out,
               const double* force, double t0, int nsteps);

/* the interface reconstruction of Eq. (gradient) on its own (for tests):
 * f-bar(x_b, t_n + h) on every interface of one axis, before wall rules,
 * from given f-bar-plus values phi[q][cells] at the cell centres (ghost
 * values by the step's extrapolation rule).  out[q][interfaces], interfaces
 * laid out [z][y][x] with n+1 along `axis` */
int oracle_interface_values(const oracle_cfg* cfg, int axis, const double* phi,
                            double* out);

/* rho, u (D comps), p at time t; each output nullable.
 * totals (nullable, 6): sum V rho, sum V j_x, sum V j_y, sum V j_z,
 * 1/2 sum V |u|^2, number of non-finite values in f */
int oracle_moments(const oracle_cfg* cfg, const double* f, const double* force,
                   double t, double* rho, double* u, double* p, double* totals);

/* reverse mode of one step (incompressible model; any mesh and boundary
 * set, walls included):
 *   lam_n      = (d f_{n+1} / d f_n)^T lam_np1
 *   grad_force += (d f_{n+1} / d force)^T lam_np1   (nullable) */
int oracle_step_adjoint(const oracle_cfg* cfg, const double* f_n, const double* force,
                        double t_n, const double* lam_np1, double* lam_n,
                        double* grad_force);

/* reverse mode of oracle_init with rho = rho0 everywhere:
 *   grad_u     += (d f0 / d u)^T lam0       (nullable)
 *   grad_force += (d f0 / d force)^T lam0   (nullable) */
int oracle_init_adjoint(const oracle_cfg* cfg, const double* u, const double* force,
                        double t0, const double* lam0, double* grad_u, double* grad_force);

/* number of OpenMP threads the oracle uses */
int oracle_threads(void);

#ifdef __cplusplus
}
#endif
#endif
