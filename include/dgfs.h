/*
 * dgfs.h -- C ABI of the MI355X (gfx950) multi-species fast Fourier spectral
 * collision operator.
 *
 * The library evaluates, for a batch of independent spatial points ("nodes"),
 *
 *     Q^i(v) = sum_j Q^{ij}(f^i, f^j)(v),        i = 1..s,
 *
 * the right-hand side of the dimensionless multi-species Boltzmann equation
 * (paper: Jaiswal, Alexeenko & Hu, Sec. 3, eq. NMBE), with each Q^{ij} computed by
 * the fast spectral method of Sec. 4: Fourier series on [-L, L]^3 with N modes per
 * dimension, a Gauss-Legendre rule of n_rho points on [0, R_ij] and an M-point
 * spherical design for the gain term, and the loss term as one convolution.  The
 * per-pair constant C_ij (Kn_ij^{-1} times the kernel constant of eq. NVSS) is an
 * input, so any VHS kernel B_ij = C_ij |g|^{2(1-omega_ij)} is accepted (the fast
 * algorithm does not depend on the kernel form: the remark after eq. NVSS).
 *
 * Conventions (shared by every entry point):
 *   - Distribution functions and results are laid out [batch][s][N][N][N], the last
 *     (z) index fastest, real, in the plan's precision (float or double).
 *   - Species i is sampled at v_n = -L + n 2L/N, n = 0..N-1, per dimension (with
 *     species-specific grids, L is that species' own half-width L_i).
 *   - Mode k of the truncated series runs over [-N/2, N/2-1]^3 (Sec. 4); the DFT
 *     index N/2 stands for the mode -N/2.  The sum over l + m = k in eq. (sum) is
 *     taken modulo N (circular), which is what its FFT evaluation computes.
 *   - R_ij = 2 S with S the largest support radius allowed by the anti-aliasing
 *     condition (Sec. 4, eq. domain) for both orderings of the pair.
 *   - Spherical designs: M = 6 (octahedron), 12 (icosahedron), 24 (the orbit of
 *     one point under the 24 rotations of the cube that forms a 7-design).
 *
 * Memory and threading:
 *   - Every device pointer is owned by the caller.  The plan owns its tables,
 *     allocated on the current device in dgfs_plan_create and freed in
 *     dgfs_plan_destroy; it copies every host array of dgfs_problem.
 *   - Compute entry points are asynchronous on the given HIP stream (a
 *     hipStream_t passed as void*; NULL is the default stream) and never allocate.
 *   - A plan is immutable after creation: concurrent calls on different streams with
 *     different workspaces are allowed.
 *   - Errors are returned as dgfs_status; dgfs_last_error() gives a thread-local text.
 */
#ifndef DGFS_H
#define DGFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DGFS_OK = 0,
    DGFS_EINVAL = -1,        /* invalid argument (message in dgfs_last_error) */
    DGFS_EUNSUPPORTED = -2,  /* valid but not implemented (e.g. an N without kernels) */
    DGFS_ENOMEM = -3,        /* device allocation failed, or workspace too small */
    DGFS_EDEVICE = -4        /* a HIP call or kernel launch failed */
} dgfs_status;

enum { DGFS_FP32 = 0, DGFS_FP64 = 1 };

/* Collision kernel of one ordered pair (Sec. 2 eq. VSS, dimensionless form NVSS):
 * B_ij = prefactor * |g|^{2(1-omega)} * (1 + cos chi)^{alpha-1}, cos chi = sigma . g_hat.
 * omega in [0.5, 1]; alpha in [1, 2] (1: VHS/HS/Maxwell, > 1: variable soft spheres,
 * whose kernel mode depends on sigma: the plan then keeps one complex table per
 * direction and radial point); prefactor > 0.  The kernel must be symmetric in (i, j). */
typedef struct {
    double omega;
    double alpha;
    double prefactor;
} dgfs_pair_kernel;

typedef struct {
    int32_t s;                       /* number of species, 1..8 */
    const double* mass;              /* [s] nondimensional masses, > 0 */
    double L;                        /* half-width of the velocity box [-L, L]^3, > 0;
                                        ignored when L_species is given */
    const double* L_species;         /* NULL (every species on [-L, L]^3), or [s] half-widths
                                        L_i > 0 of species-specific grids.  Species i is then
                                        sampled at v_n = -L_i + n 2L_i/N, and the ordered pair
                                        (i, j) is evaluated by the method of Sec. 4 on the box
                                        of half-width L_ij = max(L_i, L_j) (R_ij and all tables
                                        for that box): a narrower species is carried onto it
                                        by its real trigonometric interpolant (Nyquist mode
                                        split evenly per dimension; zero outside its own box
                                        [-L_i, L_i)), and Q^{ij} is carried back to grid i by
                                        the interpolant of the L_ij grid.  The remark after
                                        eq. (domain) in Sec. 4 names such grids for large mass
                                        ratios; the carrying rule is this library's choice.
                                        The conservation correction then uses each species'
                                        own grid.  dgfs_collide_plain needs one common grid. */
    int32_t N;                       /* modes per dimension: 16, 24, 32, 48 or 64 (64: VHS kernels
                                        only; no slab, plain path or dealiased form) */
    int32_t M;                       /* spherical design size: 6, 12 or 24 */
    int32_t n_rho;                   /* radial Gauss-Legendre points, 1..128 */
    const dgfs_pair_kernel* kernel;  /* [s*s], row-major (i, j); must be symmetric:
                                        kernel[i*s+j] == kernel[j*s+i] (the cross-species
                                        conservation of Sec. 2, eq. consv, needs it) */
    int32_t precision;               /* DGFS_FP32 or DGFS_FP64 */
    int32_t tile_ch, tile_cz;        /* gain-kernel geometry: x-chunks per field and thread
                                        groups per y/z pencil; 0, 0 = the library's default
                                        for (N, precision); other values must be one of
                                        dgfs_tile_candidates (DGFS_EUNSUPPORTED otherwise).
                                        cz = 0 (with ch = 2, FP32, N = 32): the shifted fields
                                        of Sec. 4 are formed on the matrix cores as dense shift
                                        contractions with FP16 hi/lo operands and FP32 sums;
                                        VHS kernels (alpha = 1) and the circular form only, and
                                        the default for such problems. */
    int32_t dealias;                 /* 0: eq. (sum) as the circular convolution the FFT
                                        evaluation computes on the N^3 grid; 1: l + m = k
                                        taken literally (no wrap-around), evaluated with
                                        spectra zero-padded to 3N/2.  1 needs N = 16, 24, 32 or 48,
                                        alpha = 1, one common grid and the default tile. */
} dgfs_problem;

typedef struct dgfs_plan dgfs_plan;

/* The pair prefactor of the dimensionless kernel, for filling dgfs_pair_kernel: Kn_ij^{-1}
 * times the constant of the VSS kernel (Sec. 3, eqs. Kn and NVSS).  The sqrt(1 + m_i/m_j)
 * factors of the two cancel, so
 *     C_ij = alpha / (kn0 2^{1+alpha} Gamma(5/2 - omega) pi mu_ij^{omega - 1/2}),
 * mu_ij = m_i m_j / (m_i + m_j), with kn0 = 1 / (pi n0 d_ref^2 (T_ref/T0)^{omega-1/2} H0)
 * the mass-independent part of Kn_ij.  Symmetric in (m_i, m_j).  m_i, m_j, kn0 > 0,
 * omega in [0.5, 1], alpha in [1, 2] (DGFS_EINVAL otherwise); *C receives the value.
 * Host only: no device is touched. */
dgfs_status dgfs_pair_prefactor(double m_i, double m_j, double omega, double alpha, double kn0, double* C);

/* Host-side check of a problem description; no device is touched.
 * Returns DGFS_OK, DGFS_EINVAL or DGFS_EUNSUPPORTED. */
dgfs_status dgfs_check_problem(const dgfs_problem* problem);

/* Precompute (Sec. 4, the tables F and G- computed once per problem): quadrature,
 * designs, radial kernel tables F^{ij}(|k|, rho_q), loss weights G^{ij-}(|m|) and
 * phase tables, in FP64 on the host, stored in the plan precision on the current
 * device.  *out is set only on DGFS_OK. */
dgfs_status dgfs_plan_create(const dgfs_problem* problem, dgfs_plan** out);

void dgfs_plan_destroy(dgfs_plan* plan);

/* Bytes of device workspace dgfs_collide/dgfs_collide_pairs need for `batch` nodes
 * processed in one pass.  A smaller workspace (at least the one-node size) makes the
 * call process the batch in slices. */
dgfs_status dgfs_workspace_size(const dgfs_plan* plan, int64_t batch, size_t* bytes);

/* Q[b][i] = sum_j Q^{ij}(f[b][i], f[b][j]) for b < batch.
 * f, Q: device arrays [batch][s][N^3] of the plan precision; f and Q must not overlap.
 * workspace: device memory, 256-byte aligned, ws_bytes >= dgfs_workspace_size(plan, 1). */
dgfs_status dgfs_collide(const dgfs_plan* plan, const void* f, void* Q, int64_t batch,
                         void* workspace, size_t ws_bytes, void* stream);

/* Same result as dgfs_collide, for measurement: HIP events are recorded on `stream`
 * around each stage, the call waits for the work to finish, and stage_ms[0..4]
 * receives the summed durations (over batch slices) of: the forward transform of f,
 * the gain kernel (the sigma/rho loop of Sec. 4), the radial-sum and loss-spectrum
 * kernel, the x- and y-passes of the inverse transforms, and their z-pass fused with
 * the final combination.  Synchronous. */
dgfs_status dgfs_collide_timed(const dgfs_plan* plan, const void* f, void* Q, int64_t batch,
                               void* workspace, size_t ws_bytes, void* stream, float* stage_ms);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving
 * loops that must not call hipMalloc, harnesses that forbid it): dgfs_collide with a
 * workspace owned by the library instead of the caller's.  The workspace is a static
 * device array of dgfs_static_workspace_bytes() bytes (256 MiB) on every device the
 * library runs on, held until the process ends; its address is looked up once per device
 * on the first call.  The call allocates nothing; the batch runs in slices of as many
 * nodes as that workspace holds, with results equal bit for bit to dgfs_collide's.
 * f, Q: device arrays [batch][s][N^3] of the plan precision, as for dgfs_collide.  The
 * plan's device must be the current device (DGFS_EINVAL otherwise); a plan whose single
 * node needs more workspace than the array holds gives DGFS_ENOMEM.  Every call on one
 * device shares that device's array: calls that overlap on one device (other streams,
 * other host threads) race and give wrong results; serialise them. */
dgfs_status dgfs_collide_static(const dgfs_plan* plan, const void* f, void* Q, int64_t batch, void* stream);
size_t dgfs_static_workspace_bytes(void);

/* Per ordered pair: Q[b][i][j] = Q^{ij}(f[b][i], f[b][j]), Q shaped [batch][s][s][N^3]. */
dgfs_status dgfs_collide_pairs(const dgfs_plan* plan, const void* f, void* Q, int64_t batch,
                               void* workspace, size_t ws_bytes, void* stream);

/* The plain per-point FP64 path, for comparison with dgfs_collide: the same
 * discretised operator evaluated node by node with unfused kernels (for every ordered
 * pair, radial point and all M directions: phase multiply, inverse 3-D FFTs, product
 * accumulation; per radial point a forward FFT and the radial weighting; then the loss
 * convolution), without the class sharing of the antipodal designs.  Needs an FP64 plan
 * on one common grid with alpha = 1 for every pair, circular form (DGFS_EUNSUPPORTED
 * otherwise).
 * f, Q: device doubles [batch][s][N^3];
 * ws_bytes >= dgfs_workspace_size(plan, 1). */
dgfs_status dgfs_collide_plain(const dgfs_plan* plan, const double* f, double* Q, int64_t batch,
                               void* workspace, size_t ws_bytes, void* stream);

/* FP64 conservation correction (least-squares projection onto the collision
 * invariants of Sec. 2, eq. consv): with A the (s+4) x (s N^3) matrix of species
 * numbers, total momentum and total energy (rectangle rule, weight h_i^3 and m_i on
 * species i's grid),
 *     Q_out = Q_raw - A^T (A A^T)^{-1} A Q_raw      per node, in FP64.
 * Q_raw: device [batch][s][N^3] in the plan precision; Q_out: device double array of
 * the same shape (may alias Q_raw only when the plan precision is FP64). */
dgfs_status dgfs_conserve(const dgfs_plan* plan, const void* Q_raw, double* Q_out, int64_t batch,
                          void* stream);

/* One forward-Euler step of the spatially homogeneous relaxation df/dt = Q:
 *     f <- f + dt * (Q_raw - A^T (A A^T)^{-1} A Q_raw)
 * with the projection of dgfs_conserve, computed in FP64 and stored back into f in the
 * plan precision.  f, Q_raw: device [batch][s][N^3], must not overlap. */
dgfs_status dgfs_conserve_update(const dgfs_plan* plan, const void* Q_raw, void* f, double dt, int64_t batch,
                                 void* stream);

/* Time stepping of the spatially homogeneous problem df/dt = P(Q(f)), with Q the collision
 * operator of dgfs_collide and P the FP64 conservation projection of dgfs_conserve.
 * DGFS_EULER:  f <- f + dt P(Q(f)).
 * DGFS_SSPRK2: the second-order strong-stability-preserving Runge-Kutta scheme that
 *              Sec. 5 uses in time (and Sec. 6.1 for the Krook-Wu solution):
 *              f1 = f + dt P(Q(f)),  f <- f/2 + (f1 + dt P(Q(f1)))/2.
 * Each projected update is computed in FP64 and stored in the plan precision. */
enum { DGFS_EULER = 0, DGFS_SSPRK2 = 1 };

/* Bytes of device workspace dgfs_relax needs for `batch` nodes in one pass: the stage
 * states (one for Euler, two for SSP-RK2) plus the collide workspace.  A smaller
 * workspace (at least the stage states plus one node's collide workspace) makes each
 * collide run in slices. */
dgfs_status dgfs_relax_workspace_size(const dgfs_plan* plan, int64_t batch, int32_t scheme, size_t* bytes);

/* Advance f (device [batch][s][N^3], plan precision) in place by `steps` steps of size
 * dt with `scheme`.  workspace: device memory, 256-byte aligned.  Asynchronous. */
dgfs_status dgfs_relax(const dgfs_plan* plan, void* f, int64_t batch, double dt, int32_t steps, int32_t scheme,
                       void* workspace, size_t ws_bytes, void* stream);

/* ---- 1-D slab: nodal discontinuous Galerkin transport around the collision operator --
 * Sec. 5: [x0, x1] is cut into Ne equal elements with K Gauss-Lobatto-Legendre points
 * each (interpolation and quadrature points alike, so the mass matrix and the collision
 * tensor are diagonal); per element, node m, species i and velocity v
 *   dF_m/dt = 2/(h w_m) [ v_x sum_l w_l D_lm F_l - (face terms) ] + P(Q(F_m)),
 * with D_lm the derivative of the m-th Lagrange polynomial at point l and the upwind
 * flux (eq. flux) on the faces.  Outside the slab (Sec. 2): an inflow Maxwellian
 * (eq. bc_inlet) or a purely diffuse wall (eq. bc_wall with accommodation 1, its density
 * n_w from eq. bc_nwall as sums over the velocity grid).  Maxwellians are the
 * nondimensional n (m/(pi T))^{3/2} exp(-m |v - u|^2 / T) of Sec. 3.  P(Q) is the
 * collision operator of the plan followed by the FP64 projection of dgfs_conserve. */
enum { DGFS_BC_INFLOW = 0, DGFS_BC_WALL = 1 };

typedef struct {
    int32_t kind;      /* DGFS_BC_INFLOW or DGFS_BC_WALL */
    double n[8];       /* inflow: number density of each species (ignored for a wall) */
    double u[3];       /* inflow velocity, or wall velocity (its x component must be 0) */
    double T;          /* temperature, > 0 */
} dgfs_boundary;

typedef struct {
    double x0, x1;     /* ends of the slab, x1 > x0 */
    int32_t Ne;        /* elements, >= 1 */
    int32_t K;         /* GLL points per element, 2..8 */
    dgfs_boundary left, right;
    int32_t collide;   /* 1: transport and collisions; 0: transport only */
} dgfs_slab_desc;

typedef struct dgfs_slab dgfs_slab;

/* Create a slab over `plan` (not owned; it must outlive the slab).  Its state f is the
 * batch of Ne*K nodes of the plan, device [Ne][K][s][N^3] in the plan precision, node
 * (e, m) at x = x0 + e h + (1 + xi_m) h/2.  Uploads small tables to the current device. */
dgfs_status dgfs_slab_create(const dgfs_plan* plan, const dgfs_slab_desc* desc, dgfs_slab** out);
void dgfs_slab_destroy(dgfs_slab* slab);

/* Device workspace for dgfs_slab_step with `scheme` (DGFS_EULER or DGFS_SSPRK2): the
 * stage states, Q and the collide workspace for all Ne*K nodes in one pass. */
dgfs_status dgfs_slab_workspace_size(const dgfs_slab* slab, int32_t scheme, size_t* bytes);

/* Advance f in place by `steps` steps of size dt (forward Euler, or the SSP-RK2 scheme
 * of Sec. 5: f1 = f + dt L(f), f <- f/2 + (f1 + dt L(f1))/2).  workspace: device memory
 * of at least dgfs_slab_workspace_size bytes, 256-byte aligned.  Asynchronous. */
dgfs_status dgfs_slab_step(const dgfs_slab* slab, void* f, double dt, int32_t steps, int32_t scheme,
                           void* workspace, size_t ws_bytes, void* stream);

/* The slab's GLL points and weights on [-1, 1] ([K] each, host), for tests. */
dgfs_status dgfs_slab_gll(int32_t K, double* xi, double* w);

/* Host-side view of the precomputed quantities of ordered pair (i, j), for tests:
 *   info[0..5] = a, b, gamma, C_ij, R_ij, number of phase directions used;
 *   rho, w_rho: [n_rho] radial nodes and weights on [0, R_ij];
 *   loss: [3 (N/2)^2 + 1] G^{ij-} as a function of |m|^2 (no 1/N^3 factor).
 * Any output pointer may be NULL.  No device is touched. */
dgfs_status dgfs_pair_tables(const dgfs_problem* problem, int32_t i, int32_t j, double* info,
                             double* rho, double* w_rho, double* loss);

/* Host evaluation of the kernel mode of Sec. 4 (below eq. GG) for a VSS kernel, for tests:
 * F(k, rho, sigma) = rho^2 int_{S^2} C rho^gamma (1 + sigma.g_hat)^{alpha-1}
 *                    e^{-i pi rho a k.g_hat / L} dg_hat,
 * k: [3] mode vector, sigma: [3] unit vector, F: [2] real and imaginary part.  Uses the
 * same series as plan creation.  No device is touched. */
dgfs_status dgfs_kernel_mode(double alpha, double gamma, double C, double a, double L, double rho, const double* k,
                             const double* sigma, double* F);

/* Gain-kernel geometries compiled for (N, precision), as pairs (ch, cz) in
 * pairs[2*k], pairs[2*k+1], k < *count <= max_pairs; the first is the default (for VSS
 * kernels or the dealiased form: the first with cz > 0). */
dgfs_status dgfs_tile_candidates(int32_t N, int32_t precision, int32_t* pairs, int32_t max_pairs,
                                 int32_t* count);

/* ---- uneven batches: several plans (e.g. different N) evaluated together ----------
 * A group runs each plan's pipeline on its own stream, forked from and joined back to
 * the caller's stream with events, so the hardware overlaps the N-classes; a group
 * call can be captured once into a hipGraph and replayed with one launch.  The group
 * owns its streams and events (created on the current device, default priority). */
typedef struct dgfs_group dgfs_group;

dgfs_status dgfs_group_create(const dgfs_plan* const* plans, int32_t nplans, dgfs_group** out);
void dgfs_group_destroy(dgfs_group* group);

/* Bytes of one workspace covering batch[k] nodes of every plan k in one pass. */
dgfs_status dgfs_group_workspace_size(const dgfs_group* group, const int64_t* batch, size_t* bytes);

/* For every plan k: Q[k] = collide(plan k, f[k], batch[k]) (same layout as dgfs_collide).
 * The caller's stream waits for all of them.  Asynchronous. */
dgfs_status dgfs_group_collide(dgfs_group* group, const void* const* f, void* const* Q,
                               const int64_t* batch, void* workspace, size_t ws_bytes, void* stream);

/* Capture dgfs_group_collide with these arguments on `stream` (a non-default stream)
 * into a hipGraph, instantiate it and return the executable graph (hipGraphExec_t as
 * void*) in *graph.  Nothing runs during capture. */
dgfs_status dgfs_group_capture(dgfs_group* group, const void* const* f, void* const* Q,
                               const int64_t* batch, void* workspace, size_t ws_bytes, void* stream,
                               void** graph);
dgfs_status dgfs_graph_launch(void* graph, void* stream);
void dgfs_graph_destroy(void* graph);

/* Host-side copy of the M-point design used by the plan, [M][3]. */
dgfs_status dgfs_design(int32_t M, double* sigma);

/* Host-side copy of the one-dimensional map between species grids used with
 * L_species, for tests: T[r*N + n] weights sample n of the grid of half-width L_from to
 * give the real trigonometric interpolant at point r of the grid of half-width L_to
 * (zero rows for points outside [-L_from, L_from)); the three-dimensional map applies T
 * along each axis.  T: [N][N] host doubles.  No device is touched. */
dgfs_status dgfs_interpolation_matrix(int32_t N, double L_from, double L_to, double* T);

/* Measurement aid: the attainable FP32 vector FMA rate of the current device (the
 * ceiling the kernels' arithmetic can reach, stated beside the datasheet peak).  Runs
 * `blocks` workgroups of 256 threads, each thread `iters` x 8 independent FMAs, once to
 * warm up and once timed with HIP events on `stream` (synchronous).  scratch: device
 * memory of at least blocks * 256 floats.  *tflops receives the measured rate. */
dgfs_status dgfs_probe_valu(void* scratch, size_t scratch_bytes, int32_t blocks, int32_t iters, void* stream,
                            double* tflops);

const char* dgfs_status_string(dgfs_status status);
const char* dgfs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DGFS_H */
