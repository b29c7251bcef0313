/*
 * dugks.h -- C ABI of the MI355X (gfx950) incompressible-DUGKS library.
 *
 * One time step of the incompressible discrete unified gas-kinetic scheme
 * with body force of Wu, Shi, Chai & Wang (arXiv:1411.6121), its adjoint,
 * and a batched form, for the D2Q9, D3Q19 and D3Q27 velocity sets on uniform and
 * tanh-stretched Cartesian meshes.  Every stage runs in hand-written HIP
 * kernels; this header is the whole interface.
 *
 * Conventions shared by all entry points
 * --------------------------------------
 * Data layout (all device arrays are dense, C-contiguous, 256-byte aligned
 * is recommended, element type = the context dtype):
 *   distribution state  f[q][z][y][x]   x fastest, Q = 9 or 19 planes
 *   vector field        v[d][z][y][x]   d < D (2 or 3 components)
 *   scalar field        s[z][y][x]
 * For D2Q9, nz = 1.  Velocity order (e = (ex, ey, ez) in {-1,0,1}^3):
 *   D2Q9  : ex outer, ey inner (the order printed in Sec. II.C);
 *           rest state at q = 4, opposite of q is 8 - q.
 *   D3Q19 : ex outer, ey middle, ez inner, dropping the 8 corners
 *           |e|^2 = 3; rest state at q = 9, opposite of q is 18 - q;
 *           weights 1/3 (rest), 1/18 (|e|^2 = 1), 1/36 (|e|^2 = 2).
 *   D3Q27 : the paper's 3-D set: ex outer, ey middle, ez inner, all 27;
 *           rest state at q = 13, opposite of q is 26 - q; weights
 *           products of 2/3 (component 0) and 1/6 (component +-1).
 *   Discrete velocities xi_q = sqrt(3 RT) e_q (Sec. II.C).
 * The stored state is f-tilde = f - dt/2 Omega - dt/2 S (Sec. II.B).
 *
 * Ownership: every state, field and output buffer is caller-owned device
 * memory; the library never allocates or frees it.  A context owns only
 * its small metric/coefficient tables and the per-launch scratch it
 * documents below.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = default
 * stream).  Calls are asynchronous on that stream unless documented as
 * synchronising.
 *
 * Errors: every int-returning call returns DUGKS_OK (0) or a negative code;
 * the message of the last failure of a context is dugks_last_error(ctx),
 * of a failed dugks_init is dugks_last_error(NULL).  Asynchronous HIP
 * errors surface at the next synchronising call as DUGKS_EHIP.
 *
 * Threading: one context per host thread at a time; calls that overlap on
 * one context race.
 *
 * Determinism: the forward path uses no atomics; results are bitwise
 * reproducible from run to run on the same device.
 */
#ifndef DUGKS_H
#define DUGKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DUGKS_OK 0
#define DUGKS_EINVAL (-1)       /* invalid argument or configuration        */
#define DUGKS_EUNSUPPORTED (-2) /* valid but not implemented for this case  */
#define DUGKS_EHIP (-3)         /* HIP runtime error                        */
#define DUGKS_ENONFINITE (-4)   /* moments found NaN/Inf in the state       */
#define DUGKS_ENOMEM (-5)       /* device allocation of context tables      */

enum dugks_lattice { DUGKS_D2Q9 = 9, DUGKS_D3Q19 = 19, DUGKS_D3Q27 = 27 };
enum dugks_dtype { DUGKS_F32 = 0, DUGKS_F64 = 1 };
/* mesh of one axis: uniform, the tanh stretching of Eq. (Nonuniform_mesh),
 * or caller-given face coordinates (dugks_config.faces) */
enum dugks_mesh_kind { DUGKS_UNIFORM = 0, DUGKS_TANH = 1, DUGKS_CUSTOM = 2 };
/* equilibrium model: the paper's incompressible one (Eq. icfeq with
 * Eq. macro_values) or the original DUGKS one (Eq. feq with
 * rho u = sum xi f + rho G dt/2), kept for comparison */
enum dugks_model { DUGKS_MODEL_INCOMPRESSIBLE = 0, DUGKS_MODEL_ORIGINAL = 1 };
/* boundary kinds, one per domain side (-x,+x,-y,+y,-z,+z) */
enum dugks_bc {
    DUGKS_PERIODIC = 0,     /* both sides of the axis must be periodic      */
    DUGKS_NEQ_VELOCITY = 1, /* Eq. (NEQ), velocity condition u_w           */
    DUGKS_NEQ_PRESSURE = 2, /* Eq. (NEQ), pressure condition p_w           */
    DUGKS_BOUNCE_BACK = 3   /* Eq. (BB), wall velocity u_w, rho_w = rho0    */
};

/*
 * Problem description (Sec. II; mesh of Eq. Nonuniform_mesh).
 *   n[3]        cells per axis (n[2] = 1 for D2Q9); wall axes need n >= 2
 *   L[3]        domain length per axis
 *   mesh[3]     DUGKS_UNIFORM, DUGKS_TANH or DUGKS_CUSTOM per axis; faces of
 *               a tanh axis are X_i = L (1/2 + tanh(k (i/N - 1/2)) / (2 tanh(k/2)));
 *               a custom axis takes faces[a]
 *   faces[3]    per axis, for DUGKS_CUSTOM only (else ignored, may be NULL):
 *               host array of the n[a]+1 face coordinates, X_0 = 0 <
 *               X_1 < ... < X_n = L[a] exactly (a finite-volume mesh as in
 *               Sec. II.B and the Appendix, cell widths X_{i+1} - X_i,
 *               centres at the midpoints); read by dugks_init and
 *               dugks_batch_create, which keep their own copies
 *   rho0, RT    reference density, R T (c = sqrt(3 RT))
 *   tau, dt     relaxation time and time step (both > 0)
 *   G[3]        uniform part of the acceleration
 *   omega,phase acceleration time factor g(t) = cos(omega t + phase):
 *               G(x, t) = g(t) (G + G^(x)), G^ the optional force field
 *   bc[6]       side kinds; uw[6][3] wall velocities; pw[6] wall pressures
 *               (pressure p = (rho - rho0) RT)
 *   model       DUGKS_MODEL_INCOMPRESSIBLE (0, the paper's model) or
 *               DUGKS_MODEL_ORIGINAL (1: the two-lane fused kernel where the
 *               incompressible model would take it and no force field is
 *               given, else the general kernels; no batched form, no
 *               adjoint: DUGKS_EUNSUPPORTED there)
 *   pw_osc[6]   oscillating part of the wall pressures: a pressure side
 *               holds p_w(t) = pw[s] + pw_osc[s] g(t), with g the time
 *               factor above taken at the interface time t_n + dt/2 of
 *               the step (the pressure-driven flow of Sec. III.C, whose
 *               inlet pressure follows Eq. Wom_AS_Pressure); zero for a
 *               constant pressure.  rho0 + (pw - |pw_osc|) / RT must stay
 *               positive.
 * D3Q27 has no batched form and no adjoint (DUGKS_EUNSUPPORTED).
 */
typedef struct {
    int lattice;
    int dtype;
    int n[3];
    double L[3];
    int mesh[3];
    double k_stretch;
    double rho0, RT, tau, dt;
    double G[3];
    double omega, phase;
    int bc[6];
    double uw[6][3];
    double pw[6];
    int model;
    const double* faces[3];
    double pw_osc[6];
} dugks_config;

typedef struct dugks_ctx dugks_ctx;
typedef struct dugks_batch dugks_batch;

/* Library version string. */
const char* dugks_version(void);

/* Message of the last failure on ctx (NULL: the last failed dugks_init /
 * dugks_batch_create on this thread).  Never NULL. */
const char* dugks_last_error(const dugks_ctx* ctx);

/* dt = cfl * (smallest cell width) / sqrt(3 RT)  (Sec. III, CFL condition).
 * Returns a negative value for an invalid configuration. */
double dugks_dt_from_cfl(const dugks_config* cfg, double cfl);

/*
 * Create a context and write the initial state (the runs of Sec. III start
 * from equilibrium): f~0 = feq(rho, u) - dt/2 S(rho, u, G(x, t0)) with the
 * incompressible equilibrium of Eq. (icfeq) and S of Eq. (S), i.e. the
 * state whose original distribution is the equilibrium.
 *   rho    nullable scalar field (NULL: rho0 everywhere)
 *   u      nullable vector field [D] (NULL: rest)
 *   force  nullable force field G^ [D] (NULL: zero)
 *   f_out  state buffer [Q] written on `stream`
 *   out    receives the context; on failure *out = NULL and the error is
 *          readable with dugks_last_error(NULL)
 * t0 = 0.  The context owns device tables of O(n) size and, for the
 * general kernels, one scratch state of (n+2)^D Q elements.
 */
int dugks_init(const dugks_config* cfg, const void* rho, const void* u, const void* force,
               void* f_out, void* stream, dugks_ctx** out);

/* Write the initial state of the context's configuration at time t0 again
 * (same arguments as dugks_init). */
int dugks_reset(dugks_ctx* ctx, const void* rho, const void* u, const void* force, double t0,
                void* f_out, void* stream);

/*
 * One time step t_n -> t_n + dt of the scheme (Sec. II.B and the Appendix):
 * f-bar-plus at the centres (Eq. f_bar_+), ghost extrapolation, interface
 * reconstruction f-bar(x_b, t_n+h) = f-bar-plus(x_b) - xi h . grad
 * (Eq. gradient), wall rules (Eqs. BB, NEQ), interface moments, original
 * distribution at the interface (inverse of Eq. original_f), micro-flux
 * (Eq. microflux) and the conservative update (Eqs. f_tilde_+,
 * evolution_equation).
 *   f_in, f_out  distinct state buffers [Q] (ping-pong; f_in == f_out is
 *                DUGKS_EINVAL)
 *   force        nullable force field G^ [D]
 *   t_n          time of f_in (enters only through g(t))
 * Asynchronous on `stream`.
 */
int dugks_step(dugks_ctx* ctx, const void* f_in, void* f_out, const void* force, double t_n,
               void* stream);

/* nsteps steps from f_a at time t0, ping-ponging between f_a and f_b;
 * *which_out = 0 if the result is in f_a, 1 if in f_b.  Asynchronous. */
int dugks_run(dugks_ctx* ctx, void* f_a, void* f_b, const void* force, double t0, int nsteps,
              void* stream, int* which_out);

/*
 * Macroscopic fields at time t (Eq. macro_values):
 *   rho = sum_q f~_q, u = sum_q xi_q f~_q / rho0 + dt/2 G(x, t),
 *   p = (rho - rho0) RT.  rho, u [D], p are nullable device outputs.
 * totals_host (nullable, 6 doubles, host memory): sum V rho, sum V j_x,
 * sum V j_y, sum V j_z (j = sum xi f~), 1/2 sum V |u|^2, count of
 * non-finite values in f.  With totals_host the call synchronises `stream`
 * and returns DUGKS_ENONFINITE if the count is non-zero.  The reduction is
 * deterministic (fixed-order two-pass, no atomics).
 */
int dugks_moments(dugks_ctx* ctx, const void* f, const void* force, double t, void* rho, void* u,
                  void* p, double* totals_host, void* stream);

/*
 * The six totals of dugks_moments (mass, momentum, kinetic energy E_k =
 * 1/2 int |u|^2 dx, count of non-finite values) written to device memory
 * totals_dev[0..5] (8-byte aligned, caller-owned) in stream order, without
 * synchronising and without a host copy: calling it every k steps with
 * successive slots records the E_k history of Sec. III on the device (and
 * inside a captured graph).  Uses the context's reduction scratch: calls on
 * one context go on one stream.  Non-finite values are reported in slot 5,
 * not as an error.
 */
int dugks_totals_async(dugks_ctx* ctx, const void* f, const void* force, double t, double* totals_dev,
                       void* stream);

/*
 * Convergence monitor of Sec. III (the steady criterion of the periodic
 * flow, the periodic criterion of the Womersley flow): with u_a, u_b the
 * velocities of Eq. (macro_values) of the states f_a at time t_a and f_b
 * at time t_b (force field as in dugks_moments, nullable),
 *   out_host[0] = sqrt(sum over cells |u_b - u_a|^2),
 *   out_host[1] = sqrt(sum over cells |u_b|^2),
 * unweighted sums as in the paper; the criterion is their ratio (for
 * example below 1e-6 with t_b = t_a + 1000 dt).  The kinetic-energy
 * history E_k = 1/2 int |u|^2 dx is totals[4] of dugks_moments.
 * Deterministic reduction; uses the context's reduction scratch, so calls
 * on one context must not overlap.  Synchronises the stream;
 * DUGKS_ENONFINITE if either state holds a non-finite velocity.
 */
int dugks_velocity_change(dugks_ctx* ctx, const void* f_a, const void* f_b, const void* force, double t_a,
                          double t_b, double* out_host, void* stream);

/*
 * Reverse mode of one step (the scheme of Sec. II.B transposed, incompressible
 * model, D2Q9 and D3Q19) on any mesh and boundary set: periodic sides,
 * bounce-back (Eq. BB) and NEQ velocity/pressure walls (Eq. NEQ), uniform
 * or tanh-stretched axes:
 *   lam_n       = (d f_{n+1} / d f_n)^T lam_np1
 *   grad_force += (d f_{n+1} / d G^)^T lam_np1   (nullable, [D])
 * The forward intermediates are recomputed from f_n (no tape).  Fully
 * periodic meshes take a gather form: in 2-D two launches over cell tiles
 * (f-bar-plus and the interface adjoints; then the cell adjoints, the
 * neighbours' terms staged in LDS), in 3-D four passes; meshes with walls a
 * gather form over every face and the ghost-extended grid (the ghost rule
 * of the ghost values is transposed).  The scratch (2-D periodic: D (Q + D) values per
 * cell; otherwise about (2 + D) Q values per extended cell plus (Q + D) per
 * face and per cell) is allocated on first use and kept by the context.  lam_n must not alias f_n or lam_np1.  The original-model
 * variant and D3Q27 return DUGKS_EUNSUPPORTED.  Asynchronous.
 */
int dugks_step_adjoint(dugks_ctx* ctx, const void* f_n, const void* force, double t_n,
                       const void* lam_np1, void* lam_n, void* grad_force, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight loops, harnesses that forbid hipMalloc): the same
 * operation, arguments and results as dugks_step_adjoint, with the scratch
 * taken from a static device area of 64 MiB (each GPU the library runs on
 * holds it until the process ends) instead of the context's lazily
 * allocated buffer.  The call allocates and frees nothing.  The caller still
 * owns every input and output.  A problem whose scratch exceeds 64 MiB is
 * rejected with DUGKS_EINVAL (the message states both sizes; 64 MiB holds
 * the 256^2 D2Q9 FP64 adjoint, periodic or with walls).  The current device
 * must be the one the context was created on.  Every call on one GPU
 * shares that GPU's area and every element the kernels read is written
 * earlier in the same call, so nothing needs clearing; calls that overlap
 * on one GPU (other streams, other threads, other contexts) race.
 * Asynchronous.
 */
int dugks_step_adjoint_static(dugks_ctx* ctx, const void* f_n, const void* force, double t_n,
                              const void* lam_np1, void* lam_n, void* grad_force, void* stream);

/*
 * Reverse mode of the initial state with rho = rho0:
 *   grad_u     += (d f0 / d u)^T lam0   (nullable, [D])
 *   grad_force += (d f0 / d G^)^T lam0  (nullable, [D])
 * at time t0.  Asynchronous.
 */
int dugks_init_vjp(dugks_ctx* ctx, const void* u, const void* force, double t0, const void* lam0,
                   void* grad_u, void* grad_force, void* stream);

/* Which step kernel a launch without a force field uses (diagnostics):
 * 0 = general two-pass kernels, 1 = fused single launch with every
 * interface evaluated by both neighbouring cells, 2 = fused single launch
 * with every interface evaluated once, 3 = as 2 with the velocity set split
 * over two lanes per column.  By default each launch takes the faster one
 * on MI355X: 3 for D2Q9 and D3Q27, for D3Q19 FP64 without a force field
 * and for D3Q19 FP32 on uniform meshes without one; 2 otherwise.  The
 * original-model variant uses 3 where the incompressible model would and
 * no force field is given, else 0.  A batch decides
 * once for all its instances (uniform meshes, any force field), so batched
 * and single-instance states are bitwise equal when the instances share
 * the mesh kind and the presence of a force field.  All kernels give the
 * same results to rounding. */
int dugks_kernel_variant(const dugks_ctx* ctx);

/*
 * Reverse mode of the read-out of dugks_moments at time t:
 *   lam[q]      = grad_rho + xi_q . grad_u / rho0     (overwritten, [Q])
 *   grad_force += g(t) dt/2 grad_u                      (nullable, [D])
 * grad_rho (scalar field) and grad_u ([D]) are nullable (= zero).
 * Asynchronous.
 */
int dugks_moments_vjp(dugks_ctx* ctx, const void* grad_rho, const void* grad_u, double t, void* lam,
                      void* grad_force, void* stream);

/* Release the context and its device tables (synchronises its stream). */
void dugks_destroy(dugks_ctx* ctx);

/* ---------------------------------------------------------------------- */
/* batched instances                                                       */
/* ---------------------------------------------------------------------- */
/*
 * Many independent problems of uneven size, viscosity and forcing advanced
 * by one kernel launch per step.
 *   cfgs[n]     configurations (same lattice and dtype for all)
 *   offsets[n]  element offset of instance i's state inside the packed
 *               state buffer (each instance's Q planes are contiguous at
 *               that offset, in the single-instance layout)
 * The batch owns an instance table and its metric tables.
 */
int dugks_batch_create(const dugks_config* cfgs, int n, const int64_t* offsets, void* stream,
                       dugks_batch** out);

/* Initial state of every instance at time 0: the equilibrium at rest at
 * rho0 under its uniform acceleration G (force fields enter from the first
 * step); resets the batch clock. */
int dugks_batch_init(dugks_batch* b, void* f_out, void* stream);

/*
 * nsteps steps of every instance from f_in.  Steps ping-pong between f_in
 * and f_out; after an odd nsteps the result is in f_out, after an even
 * nsteps in f_in (*which_out = 1 or 0).  The batch keeps a device-side step
 * counter s (0 after dugks_batch_init, +nsteps per run): instance i is at
 * time s dt_i, so time-dependent forcing stays correct across runs.
 * Instance i uses the force field forces + force_offsets[i] when forces is
 * non-NULL and force_offsets[i] >= 0 (force_offsets nullable = no fields).
 * With use_graph != 0 the launches are captured once into a hipGraph (per
 * buffer pair, force buffer and nsteps) and replayed; this needs a
 * non-default stream.  Asynchronous.
 */
int dugks_batch_run(dugks_batch* b, void* f_in, void* f_out, const void* forces,
                    const int64_t* force_offsets, int nsteps, int use_graph, void* stream,
                    int* which_out);

/* dugks_batch_run with the launch form chosen by the library: replayed
 * from a captured hipGraph when stream is a non-default stream (graphs need
 * one), plain launches on the default stream; tile and chunk from the
 * batch's tuning (dugks_batch_tune), else the chunk model.  Same arguments,
 * results and ping-pong convention as dugks_batch_run. */
int dugks_batch_step(dugks_batch* b, void* f_in, void* f_out, const void* forces,
                     const int64_t* force_offsets, int nsteps, void* stream, int* which_out);

/*
 * Autotuner of the batched launch: times nsteps steps (after one warm-up
 * step) for every tile shape of the lattice (D3Q19: 18 x 14 columns; D2Q9:
 * rows of 128, 64 or 256 columns) and every chunk policy: each instance's
 * own march chunk from the chunk model (the device's resident workgroups
 * shared among the instances in proportion to their cells; chunk 0, also
 * the batch's default), or one chunk of 4, 8, 16, 32 or 64 planes for all,
 * and keeps the fastest for later dugks_batch_run calls.  Results do not
 * depend on the choice (every interface is evaluated by the same code in
 * any tiling), so tuning never changes a state.
 *   f_a, f_b   two distinct caller-owned scratch buffers of the batch's
 *              size, holding a valid state (e.g. copies of the current
 *              one); both are overwritten
 *   forces, force_offsets  as in dugks_batch_run (the tuned workload)
 *   tile_out, chunk_out    nullable: the chosen tile variant and chunk
 *                          policy (0 = per-instance chunks)
 * Synchronises the stream; the batch clock is left unchanged.  Drops any
 * captured graph.  DUGKS_EINVAL for bad arguments or nsteps < 1.
 */
int dugks_batch_tune(dugks_batch* b, void* f_a, void* f_b, const void* forces, const int64_t* force_offsets,
                     int nsteps, void* stream, int* tile_out, int* chunk_out);

void dugks_batch_destroy(dugks_batch* b);

/* Message of the last failure on b (NULL: the last failed
 * dugks_batch_create on this thread).  Never NULL. */
const char* dugks_batch_last_error(const dugks_batch* b);

#ifdef __cplusplus
}
#endif
#endif
