/*
 * sfac.h - C ABI of the MI355X (gfx950) library for the two-level Strang splitting of the
 * 2D/3D spatial fractional Allen-Cahn equation
 *
 *     u_t = eps^2 L^alpha u + u - u^3   on [a,b]^d, homogeneous Dirichlet boundary,
 *
 * (Cai, Fang, Chen, Sun, arXiv 2209.08437). One step of the method, eq. (finalstrang):
 *
 *     u <- J^Q_{tau/2} ( e^{tau/2 C_a} e^{tau S_a} e^{tau/2 C_a} ) J^Q_{tau/2} u,
 *
 * where J^Q_t v = v / sqrt(v^2 + (1 - v^2) e^{-2t}) is the closed-form nonlinear flow of
 * eq. (nonlinear_operator), and C_a, S_a are the Kronecker sums of the per-axis circulant and
 * skew-circulant parts of the symmetric Toeplitz matrix B_alpha (eqs. (B), (C), (S), Sec. 2.1-2.2).
 * Each exponential is applied along every axis with fast Fourier transforms (Remark 1).
 *
 * Conventions shared by every entry point
 *  - Axis 1 is the paper's x^(1) (index i), the fastest-varying index of the state vector
 *    (Sec. 2.1). A state of d axes is a dense C-order array of shape (N_d, ..., N_1) holding
 *    the interior nodes only; the Dirichlet zeros are implicit.
 *  - N_l is the number of interior nodes on axis l (the paper's m_l - 1); h_l its mesh width.
 *  - Device pointers are HIP device addresses owned by the caller; the library never frees
 *    them. Host pointers are read during the call only.
 *  - Every call returns a status; nothing throws across the ABI. On a non-OK status
 *    sfac_last_error() returns a thread-local message describing it.
 *  - A plan or batch is not reentrant: calls on one handle must not overlap. Distinct
 *    handles may be used from different threads.
 */
#ifndef SFAC_H
#define SFAC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SFAC_OK = 0,
    SFAC_EINVAL = 1,       /* an argument is outside its documented range */
    SFAC_EUNSUPPORTED = 2, /* valid, but beyond what this library implements (e.g. N too large) */
    SFAC_ENOMEM = 3,       /* a device or host allocation failed */
    SFAC_EDEVICE = 4,      /* a HIP runtime call failed; the message carries its text */
    SFAC_EBUDGET = 5       /* a request does not fit the caller's device-memory budget */
} sfac_status;

typedef enum { SFAC_FP64 = 0, SFAC_FP32 = 1 } sfac_dtype;

/* How one axis applies its circulant / skew-circulant exponentials (both exact, they differ
 * only in rounding):
 *  SFAC_METHOD_DIAG:  Remark 1 literally. e^{tC} x = F^-1 diag(e^{t lambda}) F x and
 *                     e^{tS} x = conj(psi) . F^-1 diag(e^{t mu}) F (psi . x) with length-N
 *                     mixed-radix transforms and psi_k = e^{-i pi k / N}. Needs every prime
 *                     factor of N to be at most 31.
 *  SFAC_METHOD_EMBED: the same circulant and skew-circulant matrices are symmetric Toeplitz;
 *                     each is applied as a linear convolution by its first column, computed
 *                     with one forward and one inverse length-M transform, M = 2^k >= 2N - 1.
 *                     Works for every N.
 *  SFAC_METHOD_AUTO:  the library picks per axis (the faster of the two for N and dtype).
 *  SFAC_METHOD_EXACT: not the two-level scheme but the one-level scheme of eq. (strang), the
 *                     one the paper compares with (Tables 2 and 4): the whole linear step is
 *                     e^{tau A}, A the Kronecker sum of the axes' matrices B of eq. (B), applied as
 *                     one dense product per axis with e^{tau B} (computed once in FP64 on the
 *                     host, see sfac_exact_exponential). O(N) work per point and axis instead of
 *                     O(log N): a reference scheme, not a fast path. Every axis of the plan must
 *                     ask for it; SFAC_FP64 only; N_l <= 1024; single plans only (not groups or
 *                     batches); kernel, elems_log2 and lines_per_block are ignored.
 * Precision: SFAC_FP64 plans apply each factor K as written. SFAC_FP32 plans apply it in
 * increment form, x + (K - I) x, with tables of K - I (expm1 of the eigenvalue exponents): the
 * same operator, but the transforms round the increment instead of the state, which keeps the
 * error of long FP32 runs near the single-step rounding of smooth states. */
typedef enum {
    SFAC_METHOD_AUTO = 0,
    SFAC_METHOD_DIAG = 1,
    SFAC_METHOD_EMBED = 2,
    SFAC_METHOD_EXACT = 3
} sfac_method;

/* sfac_axis_tables flag: the increment-form tables (of K - I) that SFAC_FP32 plans use. */
#define SFAC_TABLES_INCREMENT 0x100

typedef struct sfac_plan_s* sfac_plan;
typedef struct sfac_batch_s* sfac_batch;

/* Optional plan settings; pass NULL for the defaults. Zero-initialised fields mean "default". */
typedef struct {
    int32_t method[3];          /* sfac_method per axis (axis 1 first); default SFAC_METHOD_AUTO */
    int32_t use_graph;          /* 1 (default): replay steps from captured HIP graphs; 0: plain launches */
    int32_t graph_chunk;        /* steps captured per graph replay (default 32, 1..1024); sfac_step
                                   replays that graph nsteps / graph_chunk times and graphs of
                                   1, 2, 4, .. steps for the remainder (one per set bit) */
    int32_t elems_log2[3];      /* embedded method: log2 of the elements each thread holds, 2, 3 or 4
                                   (0 = automatic; 2 only for transform lengths 64..2048); fewer
                                   elements means more threads per line */
    int32_t lines_per_block[3]; /* pairs of real lines per thread block (0 = automatic) */
    int32_t kernel[3];          /* 0 automatic. Diagonal method: 1 the generic kernel (every N whose
                                   prime factors are <= 31), 2 the register-resident two-step kernel
                                   (N = A B for the pairs it is built for; SFAC_EUNSUPPORTED else),
                                   3 the same kernel with lines aligned to wavefronts (floor(64/P)
                                   lines of P = max(A, B) threads each; exchanges need no
                                   workgroup barrier; lines_per_block counts lines as before).
                                   1-3 select the diagonal method under SFAC_METHOD_AUTO and are
                                   SFAC_EINVAL with SFAC_METHOD_EMBED.
                                   Embedded method: 4 the tile is loaded and stored through LDS,
                                   adjacent threads on adjacent memory (on a strided axis, adjacent
                                   line pairs at one position), with at least two line pairs per
                                   block by default; for transform lengths >= 64
                                   (SFAC_EUNSUPPORTED else). 4 selects the embedded method under
                                   SFAC_METHOD_AUTO and is SFAC_EINVAL with SFAC_METHOD_DIAG */
} sfac_options;

/* Per-plan sticky status, read with sfac_plan_flags. */
#define SFAC_FLAG_NONFINITE 1u  /* a NaN or infinity was stored */
#define SFAC_FLAG_ABOVE_ONE 2u  /* some |u| > 1 was stored (the discrete maximum principle,
                                   Theorem 1, says this does not happen when |u0| <= 1) */

/*
 * sfac_plan_create - build the per-axis tables of eqs. (g_coe), (omega_coe), (B), (C), (S)
 * and Remark 1 in FP64 on the host, upload them, and prepare the step launches.
 *   out        : receives the plan; *out = NULL on failure.
 *   dims       : number of axes, 1, 2 or 3 (the paper treats 2 and 3; 1 is accepted).
 *   n_axis     : dims values N_l >= 1, axis 1 first.
 *   alpha_axis : dims fractional orders, each in (1, 2] (alpha = 1 makes cos(alpha pi/2) = 0;
 *                the paper uses (1, 2), alpha = 2 is the three-point Laplacian).
 *   eps        : interface parameter, >= 0 (the paper uses eps > 0; 0 gives the pure ODE).
 *   tau        : time step, > 0.
 *   h_axis     : dims mesh widths h_l = (b - a)/(N_l + 1) > 0.
 *   dt         : arithmetic of the state and of every kernel (tables are always built in FP64
 *                and rounded once for SFAC_FP32).
 *   hip_stream : hipStream_t the steps are ordered on; NULL means the legacy default stream.
 *   opt        : NULL or settings as above.
 * Errors: SFAC_EINVAL for arguments out of range or SFAC_METHOD_EXACT on some axes only,
 * SFAC_EUNSUPPORTED for N_l above 4096 (diagonal method), 2048 (embedded method) or 1024 (exact
 * exponential), or SFAC_METHOD_EXACT with SFAC_FP32, SFAC_ENOMEM, SFAC_EDEVICE.
 * A plan of SFAC_METHOD_EXACT also holds a state-sized FP64 scratch buffer (the per-axis
 * products alternate between it and the state).
 */
sfac_status sfac_plan_create(sfac_plan* out, int32_t dims, const int32_t* n_axis,
                             const double* alpha_axis, double eps, double tau,
                             const double* h_axis, sfac_dtype dt, void* hip_stream,
                             const sfac_options* opt);

/*
 * sfac_step - advance the state by nsteps steps of eq. (finalstrang), in place.
 *   u_dev  : device pointer to prod(N_l) values of the plan's dtype, C-order (N_d, .., N_1),
 *            aligned to the element size.
 *   nsteps : >= 0; 0 returns at once.
 * Asynchronous on the plan's stream: it returns once the work is queued.
 * Axis order: the per-axis factors commute (C_a and S_a are Kronecker sums over the axes, Sec.
 * 2.2), so the passes of a step may run in any axis order. Steps alternate between the orders
 * 1..d and d..1 by the parity of the number of steps the plan has queued (through sfac_step
 * and groups alike), which makes the last pass of a step and the first of the next cover the
 * same axis; one launch does both, the step boundary (closing J^Q_{tau/2}, statistics, opening
 * J^Q_{tau/2}) applied in registers, bitwise as the two launches would give it (a plan of
 * SFAC_METHOD_EXACT likewise applies one step's closing half-step and the next one's opening
 * half-step in one launch). Splitting a run into several calls, graph chunks or plain launches,
 * and stepping through a group, give bitwise the same result as one call.
 * Errors: SFAC_EINVAL (NULL plan or pointer, misaligned pointer, nsteps < 0), SFAC_EDEVICE.
 */
sfac_status sfac_step(sfac_plan p, void* u_dev, int64_t nsteps);

/* sfac_plan_destroy - release the plan's device tables, graphs and streams; NULL is accepted.
 * Waits for the plan's queued work first. */
sfac_status sfac_plan_destroy(sfac_plan p);

/* sfac_plan_device_bytes - device memory the plan holds (tables, flags; for SFAC_METHOD_EXACT the
 * per-axis exponentials and a state-sized scratch buffer), excluding the caller's state; 0 for
 * NULL. */
size_t sfac_plan_device_bytes(sfac_plan p);

/* sfac_plan_flags - synchronize the plan's stream and read its sticky status: *flags gets
 * SFAC_FLAG_* bits, *max_abs the largest |u| stored since the last reset (either pointer may
 * be NULL). Errors: SFAC_EINVAL for a NULL plan, SFAC_EDEVICE. */
sfac_status sfac_plan_flags(sfac_plan p, uint32_t* flags, double* max_abs);

/* sfac_plan_reset_flags - clear the sticky status (queued on the plan's stream). */
sfac_status sfac_plan_reset_flags(sfac_plan p);

/*
 * sfac_plan_time_passes - measure the axis-pass kernels: for each axis, `reps` >= 1 launches of
 * that axis' pass alone on u_dev, captured into a graph and replayed once between a pair of HIP
 * events on the plan's stream; ms[0 .. dims-1] receives the mean duration per launch in
 * milliseconds (back-to-back launches, as inside the step graphs). u_dev is overwritten with
 * intermediate values: it holds no state of the scheme afterwards. Synchronizes the plan's
 * stream. For a plan of SFAC_METHOD_EXACT, `reps` whole steps run instead, with an event pair
 * around every dense product, and ms[a] is the mean duration of axis a+1's product (the
 * nonlinear half-steps run between the event pairs, untimed); the state advances by `reps`
 * steps. Errors: SFAC_EINVAL, SFAC_EDEVICE.
 */
sfac_status sfac_plan_time_passes(sfac_plan p, void* u_dev, int32_t reps, float* ms);

/*
 * sfac_plan_time_fused - measure the launches that cover an axis twice (the last pass of one
 * step and the first of the next, eq. (finalstrang) applied twice with the step boundary in
 * between; see sfac_step): `reps` >= 1 such launches on u_dev, captured into a graph and
 * replayed once between a pair of HIP events on the plan's stream. ms[0] receives the mean
 * duration per launch over axis 1 (a step in the order d..1 followed by one in the order 1..d),
 * ms[1] over axis d (the other way round), in milliseconds; 0 for an axis whose kernel does not
 * fuse (the generic diagonal kernel) and for plans of SFAC_METHOD_EXACT. For one axis both
 * entries are the same launch. u_dev is overwritten with intermediate values. Synchronizes the
 * plan's stream. Errors: SFAC_EINVAL, SFAC_EDEVICE.
 */
sfac_status sfac_plan_time_fused(sfac_plan p, void* u_dev, int32_t reps, float* ms);

/*
 * sfac_plan_energy - the discrete free energy of Sec. 5, Example 5 (the discretisation of the
 * Ginzburg-Landau functional of eq. (energy)) of the state u_dev, in the plan's layout and
 * arithmetic:
 *     E(u) = prod_l h_l * ( 1/4 sum_i (u_i^2 - 1)^2  -  1/2 u^T A u ),
 * with A the Kronecker sum over the axes of the matrices B of eq. (B) (the plan's alpha, eps, h).
 * u_dev is only read. The quadratic term is summed per axis as x^T B x over the lines, through the
 * zero-padded length-M transform of each line (M the embedded method's length, whatever method
 * the plan's passes use); sums are kept in FP64 for FP32 plans too. The first call builds the
 * kernel tables on the host and allocates them (released by sfac_plan_destroy); later calls
 * allocate nothing. Runs on the plan's stream and synchronizes it before *energy is written,
 * so it cannot be captured into a graph.
 * Errors: SFAC_EINVAL (NULL or misaligned arguments), SFAC_EUNSUPPORTED (an axis with N > 2048),
 * SFAC_ENOMEM, SFAC_EDEVICE.
 */
sfac_status sfac_plan_energy(sfac_plan p, const void* u_dev, double* energy);

/*
 * sfac_plan_trace - record the maximum norm max|u| after every step of sfac_step (the quantity
 * Sec. 5, Example 4 follows step by step; the discrete maximum principle of Theorem 1 bounds it
 * by 1). capacity > 0 allocates a record of `capacity` entries, zeroed, and restarts the step
 * count: step k (k = 0, 1, .. counted from this call) writes entry k while k < capacity, later
 * steps are counted but not recorded. capacity = 0 stops recording and frees the record. The
 * value is the same largest |u| the last pass of the step folds into sfac_plan_flags. Only
 * sfac_step records (not sfac_plan_time_passes, groups or batches). Each recorded step adds one
 * one-thread kernel to the step graphs, which this call has re-captured on the next sfac_step; a
 * plan of one axis that keeps the record launches its step boundaries unfused.
 * Synchronizes the plan's stream. Errors: SFAC_EINVAL, SFAC_ENOMEM, SFAC_EDEVICE.
 */
sfac_status sfac_plan_trace(sfac_plan p, int64_t capacity);

/*
 * sfac_plan_read_trace - synchronize the plan's stream and copy the first min(steps, record
 * capacity, `capacity`) entries of the record to out[] (host); *recorded receives the steps
 * counted since sfac_plan_trace (0 when no record is kept). out may be NULL when capacity is 0.
 * Errors: SFAC_EINVAL (NULL plan or recorded, capacity < 0, NULL out with capacity > 0),
 * SFAC_EDEVICE.
 */
sfac_status sfac_plan_read_trace(sfac_plan p, double* out, int64_t capacity, int64_t* recorded);

/* sfac_plan_method - the method (SFAC_METHOD_DIAG, SFAC_METHOD_EMBED or SFAC_METHOD_EXACT) and
 * transform length (N_l for SFAC_METHOD_EXACT) the plan uses on axis `axis` (1-based).
 * Errors: SFAC_EINVAL. */
sfac_status sfac_plan_method(sfac_plan p, int32_t axis, int32_t* method, int32_t* length);

/*
 * sfac_axis_tables - host-only introspection of the tables one axis of a plan would use (no
 * device call). For N, alpha, eps, tau, h and method (SFAC_METHOD_DIAG or SFAC_METHOD_EMBED;
 * AUTO resolves as sfac_plan_create does):
 *   *length   : transform length L (N for DIAG, M = 2^k >= 2N - 1 for EMBED);
 *   scale_c   : if not NULL, L doubles: DIAG e^{tau/2 lambda_j}/N (lambda_j = sum_k c_k
 *               e^{-2 pi i j k/N}); EMBED the length-M spectrum of the first column of
 *               e^{tau/2 C} placed as a symmetric circular kernel, divided by M;
 *   scale_s   : likewise for e^{tau S} (DIAG: mu_j = sum_k s_k e^{-i pi k (2j+1)/N});
 *   radices   : if not NULL, up to 12 stage radices, *nstages their count.
 * method | SFAC_TABLES_INCREMENT gives the tables of e^{tau/2 C} - I and e^{tau S} - I instead
 * (DIAG: expm1(tau/2 lambda_j)/N, ...; EMBED: spectra of the first columns of the factors minus
 * the identity). Call it once with NULL arrays to learn L. Errors as sfac_plan_create.
 */
sfac_status sfac_axis_tables(int32_t n, double alpha, double eps, double tau, double h, int32_t method,
                             int32_t* length, double* scale_c, double* scale_s, int32_t* radices,
                             int32_t* nstages);

/*
 * sfac_exact_exponential - host-only: the exact exponential e^{tau B} of one axis, B the
 * symmetric Toeplitz matrix of eq. (B) (N = n interior nodes, mesh width h), as the one-level
 * scheme of eq. (strang) uses it per axis (the exponential of the Kronecker sum A of the axes is
 * the Kronecker product of these). Computed in FP64 from an eigendecomposition of B (Householder
 * reduction to tridiagonal form, then implicit QR steps with the Wilkinson shift):
 * e^{tau B} = V diag(e^{tau lambda}) V^T. P receives n * n doubles, row-major (the matrix is
 * symmetric). No device call. Errors: SFAC_EINVAL (arguments as for sfac_plan_create, NULL P),
 * SFAC_EUNSUPPORTED (n > 1024).
 */
sfac_status sfac_exact_exponential(int32_t n, double alpha, double eps, double tau, double h, double* P);

/* sfac_last_error - message for the last non-OK status returned on this thread ("" if none).
 * The string stays valid until the next library call on the same thread. */
const char* sfac_last_error(void);

/* ---------------------------------------------------------------- grouped stepping
 * Several independent plans stepped together: every axis pass of every plan that needs it is
 * one launch per kernel variant (transform length and arithmetic) and pass (up to 64 plans per
 * launch), instead of one launch per plan. Used for batched solves and by the solve server's
 * continuous batching. A launch carries its plans in its kernel arguments, so a group holds no
 * device memory; the captured step graphs are kept per set of (plan, state) pairs (the 32 most
 * recently used), so repeated calls with the same plans and states replay them. A stretch of at
 * least 64 steps with a fixed set of plans replays a graph of 8 steps, the rest one step at a
 * time. */
typedef struct sfac_group_s* sfac_group;

/* sfac_group_create - a launch workspace ordered on hip_stream (NULL = legacy default stream).
 * Plans stepped through a group should be created on the same stream, so that
 * sfac_plan_flags (which synchronizes the plan's stream) sees the group's work. */
sfac_status sfac_group_create(sfac_group* out, void* hip_stream);

/*
 * sfac_group_step - advance plans[i]'s state u_dev[i] by nsteps[i] >= 0 steps, i < count. A plan
 * may appear once. Plans of both arithmetics may be mixed. Each state ends bitwise equal to
 * stepping its plan alone with sfac_step: its passes run in the axis orders its step count
 * gives them (see sfac_step), the step boundaries inside each of the group's step graphs as
 * one launch where the plan's kernel fuses (the same values as two launches), and each plan's
 * step count advances by its nsteps[i]. Asynchronous on the group's stream: it returns once the
 * work is queued and does not wait for earlier calls (dropping a cached graph when the cache is
 * full waits for the stream). The plans must stay alive until the work has run.
 * Errors: SFAC_EINVAL (NULL arguments, a repeated plan, negative steps, misaligned state),
 * SFAC_EUNSUPPORTED (a plan of SFAC_METHOD_EXACT), SFAC_ENOMEM, SFAC_EDEVICE.
 */
sfac_status sfac_group_step(sfac_group g, int32_t count, const sfac_plan* plans, void* const* u_dev,
                            const int64_t* nsteps);

/* sfac_group_destroy - waits for the group's work and frees it; NULL is accepted. */
sfac_status sfac_group_destroy(sfac_group g);

/* sfac_group_device_bytes - device memory the group itself holds: 0 (launches carry their plans in
 * their kernel arguments; the plans' own memory is counted by sfac_plan_device_bytes). */
size_t sfac_group_device_bytes(sfac_group g);

/* ---------------------------------------------------------------- batched form
 * A fixed set of independent instances (each its own dims, N, alpha, eps, tau, h) with one
 * plan each and a group to step them together. */
typedef struct {
    int32_t dims;       /* 1, 2 or 3 */
    int32_t n[3];       /* N_l, axis 1 first; unused entries ignored */
    double alpha[3];
    double eps;
    double tau;
    double h[3];
} sfac_instance_desc;

/*
 * sfac_batch_create - plan `count` instances (count >= 1) for arithmetic dt on hip_stream.
 * opts is NULL (automatic schedules) or `count` per-instance options (the kernel schedules an
 * autotuner picked; use_graph and graph_chunk are ignored). Every instance is validated as by
 * sfac_plan_create; the first invalid one fails the call with its index in the message.
 * Errors as sfac_plan_create; SFAC_EUNSUPPORTED for SFAC_METHOD_EXACT (single plans only).
 */
sfac_status sfac_batch_create(sfac_batch* out, int32_t count, const sfac_instance_desc* desc,
                              sfac_dtype dt, void* hip_stream, const sfac_options* opts);

/*
 * sfac_batch_step - advance instance i by nsteps[i] steps (>= 0) in place; u_dev[i] is its
 * state as for sfac_step. Instances with fewer steps drop out of the launches once done.
 * An instance's result is bitwise the same as stepping it alone with sfac_step.
 * Asynchronous on the batch's stream.
 * Errors: SFAC_EINVAL, SFAC_ENOMEM, SFAC_EDEVICE.
 */
sfac_status sfac_batch_step(sfac_batch b, void* const* u_dev, const int64_t* nsteps);

/* sfac_batch_plan - the plan of instance i (for sfac_plan_flags etc.), NULL if out of range.
 * It belongs to the batch: do not destroy it. */
sfac_plan sfac_batch_plan(sfac_batch b, int32_t i);

/* sfac_batch_destroy - release the batch and its plans; NULL is accepted. */
sfac_status sfac_batch_destroy(sfac_batch b);

/* sfac_batch_device_bytes - device memory the batch holds, excluding the states. */
size_t sfac_batch_device_bytes(sfac_batch b);

/* ---------------------------------------------------------------- solve without allocation
 * For callers that cannot allocate device memory (tight serving loops, harnesses that forbid
 * hipMalloc): sfac_plan_create + sfac_step + sfac_plan_flags + sfac_plan_destroy in one call that
 * allocates nothing on the device. The instance's tables and status words live in a workspace of
 * 512 KiB that the library reserves in each device's memory once (held until the process ends);
 * there is one workspace per device, shared by every call on it.
 *
 * sfac_solve_noalloc - advance u_dev by nsteps steps of eq. (finalstrang), in place, with the
 * kernels and launch order sfac_step uses (the result is bitwise that of a plan with the same
 * options), by plain launches on hip_stream.
 *   dims .. dt, hip_stream, opt : as for sfac_plan_create (use_graph and graph_chunk ignored;
 *                 SFAC_METHOD_EXACT is refused: it needs a state-sized buffer).
 *   u_dev, nsteps : as for sfac_step.
 *   flags, max_abs : if either is not NULL, the call waits for its work and writes the sticky
 *                 status of this call's steps (as sfac_plan_flags); if both are NULL the call
 *                 returns once the work is queued.
 * The tables are built on the host at every call (milliseconds for N <= 1023) and copied into the
 * workspace, ordered on hip_stream after the work already queued there. Calls that overlap on one
 * device (different streams, or different host threads without ordering) race on the workspace:
 * order them on one stream.
 * Errors: as sfac_plan_create and sfac_step; SFAC_EUNSUPPORTED when the tables of the instance need
 * more than the workspace holds (up to 192 KiB per axis: every 1D and 2D instance fits, and 3D
 * instances with N_l <= 1023; three axes of N_l = 2048 do not).
 */
sfac_status sfac_solve_noalloc(int32_t dims, const int32_t* n_axis, const double* alpha_axis, double eps,
                               double tau, const double* h_axis, sfac_dtype dt, void* u_dev, int64_t nsteps,
                               void* hip_stream, const sfac_options* opt, uint32_t* flags, double* max_abs);

#ifdef __cplusplus
}
#endif

#endif /* SFAC_H */
