/*
 * sphere_poisson.h -- C ABI of the MI355X (gfx950) DFS spectral Poisson solver.
 *
 * Method: Townsend, Wilber & Wright, "Computing with functions in spherical and
 * polar geometries I. The sphere", Section 5 ("A fast and optimal spectral
 * method for Poisson's equation").  Given samples of f on the sphere the
 * library returns samples of u with
 *
 *     sin^2(theta) u_thth + cos(theta) sin(theta) u_th + u_lamlam = sin^2(theta) f
 *
 * (eq. SphericalLaplacian) together with the integral constraint
 * int_0^pi int_-pi^pi u sin(theta) dlambda dtheta = integral
 * (eq. integralConstraint2; the paper fixes integral = 0).  The discretisation
 * is the double Fourier sphere (Section 2.2, eq. BMCsphere) with the Fourier
 * spectral method of Section 5: one banded system per lambda-wavenumber k
 * (eq. linearSystems, solved with the k^2 term subtracted), the k = 0 system
 * bordered by the integration weights of Section 4 (eq. integrationCoeffs,
 * eq. pentdiagonalPlusRankOne).
 *
 * GRID AND LAYOUT (all entry points)
 *   f, u, g, fbar are device pointers to contiguous row-major [m][n] float64
 *   arrays: element (j, i) at offset j*n + i holds the value at
 *       theta_j  = (j + 1/2) * pi / m      (colatitude, j = 0..m-1, poles excluded)
 *       lambda_i = -pi + 2 * pi * i / n    (azimuth,    i = 0..n-1).
 *   n must be even (the doubling needs lambda + pi on the grid), n >= 4,
 *   m >= 4.  Every prime factor of n/2 and of m must be <= 31.
 *   Inputs and outputs must not overlap (SP_ERR_ALIAS otherwise).
 *
 * OWNERSHIP AND STREAMS
 *   The caller owns every f/u/g/fbar buffer and the stream.  A plan owns all
 *   device workspace, twiddle tables and launch schedules; it is created once
 *   (this allocates) and may be reused for any number of solves.  Solve calls
 *   allocate nothing, enqueue their kernels on `hip_stream` (a hipStream_t;
 *   NULL = the legacy default stream) and return without waiting, unless
 *   SP_SYNC_INFO is set.  A plan must not be used by two streams at once
 *   (its workspace is shared by consecutive calls).
 *
 * BEYOND THE SOLVE (each declared below with its passage)
 *   Section 4 calculus on the same grid: tangential gradient, curl of a
 *   scalar, surface divergence, curl and vorticity, and the integral over the
 *   sphere.  Low-rank functions (Section 3, eq. lowrankRepresentation) given by
 *   factor samples: the solve of such a right-hand side, pointwise evaluation
 *   at arbitrary points, and their construction from samples by
 *   structure-preserving Gaussian elimination (which owns no plan and works in
 *   a workspace the caller provides).
 *
 * ERRORS
 *   Every function returns an sp_status; nothing is printed, thrown or
 *   aborted across this boundary.  sphere_poisson_strerror() returns a static
 *   string (for SP_ERR_HIP it includes the last HIP error text of the calling
 *   thread).
 */
#ifndef SPHERE_POISSON_H
#define SPHERE_POISSON_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SP_OK = 0,
    SP_ERR_INVALID_ARG = 1,      /* null pointer, odd or too small n, m < 4, count <= 0, bad flags */
    SP_ERR_UNSUPPORTED_SIZE = 2, /* a prime factor of n/2 or m exceeds 31, or a size exceeds 2^20 */
    SP_ERR_OOM = 3,              /* device allocation failed while planning */
    SP_ERR_HIP = 4,              /* a HIP runtime call failed (see strerror) */
    SP_ERR_NOT_CONVERGED = 5,    /* MIXED: the correction did not fall below tol; u holds the last iterate */
    SP_ERR_ALIAS = 6,            /* input and output buffers overlap */
    SP_ERR_NO_DEVICE = 7,        /* no HIP device, or the current device is not gfx950 */
    SP_ERR_BAD_PLAN = 8          /* null or destroyed plan */
} sp_status;

typedef enum {
    SP_FP64 = 0,   /* every transform and solve in float64 */
    SP_MIXED = 1   /* float32 transforms and banded solves, float64 residual, update and k = 0 system */
} sp_precision;

/* flags */
#define SP_SYNC_INFO 0x1u   /* the solve synchronises `hip_stream` and fills *info (norms computed on device) */
#define SP_AUTOTUNE 0x2u    /* plan: time candidate radix orders and row tiles for this size (cached, see below) */
#define SP_INFO 0x4u        /* MIXED: compute the info norms on the device without waiting for them;
                               sphere_poisson_get_info() reads them later */

typedef struct {
    int n_lambda;       /* n: samples in lambda (even, >= 4) */
    int m_theta;        /* m: samples in theta (>= 4) */
    int precision;      /* sp_precision */
    int max_refine;     /* MIXED: number of iterative-refinement corrections (>= 0; 1 is enough for 1e-10) */
    double tol;         /* MIXED with SP_SYNC_INFO: required ||last correction|| / ||u|| (<= 0: no check) */
    unsigned flags;     /* SP_SYNC_INFO | SP_AUTOTUNE */
    int low_k_fp64;     /* MIXED: wavenumbers k < low_k_fp64 are eliminated in float64 (their systems
                           have condition numbers near (m/k)^2, too large for float32 corrections);
                           < 0: automatic, max(16, m/64); 0 or 1: only k = 0 */
} sp_desc;

typedef struct {
    int iters;               /* refinement corrections applied (0 for FP64) */
    double rel_correction;   /* ||last correction||_2 / ||u||_2 on the grid (MIXED), 0 for FP64 */
    double f_integral;       /* quadrature of int f sin(theta) dtheta dlambda (exact for band-limited f) */
    int status;              /* sp_status of the call */
    double rel_residual;     /* MIXED: ||F - (L - k^2) X||_2 / ||F||_2 over every wavenumber's theta
                                coefficients (F: those of sin^2 f, X: those of the iterate the last
                                correction was computed from; float64), 0 for FP64 */
    double est_rel_err;      /* MIXED: estimated ||u - u_exact||_2 / ||u||_2 of the returned u, where
                                u_exact solves the discrete system: the last relative correction times
                                the contraction the corrections show (the ratio of the last two, or
                                with one correction the relative size of that correction itself, which
                                is the float32 solve's own relative error); 0 for FP64 */
} sp_info;

typedef struct sp_plan_s* sp_plan;

/* Create a plan for one (n, m, precision).  Validates sizes, factorises n/2
 * and m into radices <= 31, computes float64 twiddle tables on the host
 * (exact-angle reduction) and uploads them, allocates the spectrum workspace
 * (about 16 bytes per grid point for SP_FP64, 32 for SP_MIXED) and picks the
 * launch schedule.  `hip_stream` is used for the uploads.
 * Schedules: the radix order of the lambda and theta transforms and the rows
 * per lambda tile come from the autotuner cache when it has an entry for the
 * size (text file named by SPHERE_POISSON_TUNE_CACHE, default
 * $HOME/.cache/sphere_poisson_tune.txt), else from a fixed rule.  With
 * SP_AUTOTUNE in desc->flags (or SPHERE_POISSON_AUTOTUNE=1 in the environment)
 * missing entries are measured first: every candidate is timed with HIP events
 * on a scratch problem of the same transform length, and the fastest is kept.
 * Errors: SP_ERR_INVALID_ARG, SP_ERR_UNSUPPORTED_SIZE, SP_ERR_OOM, SP_ERR_HIP,
 * SP_ERR_NO_DEVICE.  On error *out is set to NULL. */
int sphere_poisson_plan(sp_plan* out, const sp_desc* desc, void* hip_stream);

/* Solve the Poisson problem of Section 5 for one right-hand side:
 * f (input, device, [m][n] float64), u (output, device, [m][n] float64),
 * `integral` = prescribed value of the integral of u sin(theta) over the
 * doubled-up half domain (the constraint row of the k = 0 system).
 * f is not required to have zero mean (the paper's precondition); the
 * bordered k = 0 system is solved as is and info->f_integral reports the
 * mean.  `info` may be NULL; it is filled only with SP_SYNC_INFO (or later by
 * sphere_poisson_get_info).
 * MIXED plans also use u as scratch between their kernels (the float32 first
 * iterate is kept there until the update pass overwrites it), so u holds the
 * solution only once the stream reaches the end of the solve.
 * Errors: SP_ERR_BAD_PLAN, SP_ERR_INVALID_ARG, SP_ERR_ALIAS, SP_ERR_HIP,
 * SP_ERR_NOT_CONVERGED (MIXED, SP_SYNC_INFO and tol > 0 only). */
int sphere_poisson_solve(sp_plan plan, const double* f, double* u, double integral,
                         void* hip_stream, sp_info* info);

/* The same solve for a right-hand side given in low-rank form (Section 3,
 * eq. lowrankRepresentation):
 *   f(lambda_i, theta_j) = sum_{q < rank} d[q] c[q*m + j] r[q*n + i],
 * c ([rank][m], samples of c_q at theta_j), r ([rank][n], samples of r_q at
 * lambda_i) and d ([rank]) all device float64.  The half spectrum of sin^2 f
 * in lambda is formed from the rank real DFTs of the rows of r and a rank-K
 * product (Section 4, Computation of Fourier coefficients: the coefficients
 * of a low-rank function come from 1D transforms of its factors), replacing
 * the transform of the m x n grid; the theta pass and the inverse transform
 * are those of sphere_poisson_solve, so u equals that call's result on the
 * sampled grid up to rounding.  u: output [m][n] as there (MIXED: scratch
 * until the end of the solve).  The call also uses the plan's second spectrum
 * buffer for the factor spectra (calls on one plan are stream-ordered).
 * Errors: SP_ERR_BAD_PLAN; SP_ERR_INVALID_ARG (a NULL pointer, rank < 1 or
 * rank > m); SP_ERR_ALIAS (u overlaps c, r or d); SP_ERR_HIP;
 * SP_ERR_NOT_CONVERGED as for sphere_poisson_solve. */
int sphere_poisson_solve_lowrank(sp_plan plan, int rank, const double* d, const double* c, const double* r,
                                 double* u, double integral, void* hip_stream, sp_info* info);

/* Pointwise evaluation of a low-rank function (Section 4, Pointwise
 * evaluation): out[p] = f(xyz[3p], xyz[3p+1], xyz[3p+2]) for f given as in
 * sphere_poisson_solve_lowrank (d, c, r on the plan's grid).  A point is
 * projected radially to the unit sphere: lambda = atan2(y, x),
 * theta = arccos(z / |p|) (the origin gives NaN).  The factors are
 * continued off the grid by their trigonometric interpolants with the DFS
 * even/odd structure (eq. lowrankRepresentationSplit):
 *   f = sum_q d_q (c_q^e(theta) r_q^+(lambda) + c_q^o(theta) r_q^-(lambda)),
 * c^e = sum_{s<m} alpha_s cos(s theta) and c^o = sum_{s=1..m} beta_s sin(s theta)
 * interpolating c_q at the m nodes, r^+ / r^- the even / odd wavenumbers of
 * the real Fourier interpolant of r_q (Nyquist term as a cosine); each series
 * is summed by Horner's rule, O(rank (m + n)) per point.  At the grid nodes
 * the result is the sampled f.  xyz: device [npts][3]; out: device [npts].
 * The coefficients are kept in the plan's spectrum buffers (stream-ordered
 * with the plan's other calls); computing them costs O(rank m^2).
 * Errors: SP_ERR_BAD_PLAN; SP_ERR_INVALID_ARG (a NULL pointer, npts < 0,
 * rank < 1 or rank > min(m, n/2 + 1)); SP_ERR_ALIAS (out overlaps an input);
 * SP_ERR_HIP.  npts = 0 does nothing. */
int sphere_poisson_eval_lowrank(sp_plan plan, int rank, const double* d, const double* c, const double* r,
                                int npts, const double* xyz, double* out, void* hip_stream);

/* Low-rank approximation of a sampled function by structure-preserving
 * Gaussian elimination (Section 3, Figure GaussianElimination, eq.
 * GEstructurePreservingStepPseudoinverse), on the grid f [m][n] (device,
 * float64, theta_j rows, lambda_i columns, n even).  The doubled function is
 * never formed: its value at (lambda, -theta) is the sample at
 * (lambda + pi, theta).  Step k:
 *   pivot: the grid point (theta_t, lambda_i), lambda_i in [0, pi), whose 2 x 2
 *     pivot matrix M = [[a, b], [b, a]], a = e(lambda_i - pi, theta_t),
 *     b = e(lambda_i, theta_t), has the largest sigma_1 = |a| + |b|
 *     (eq. SingularValues; ties go to the first point in row-major order);
 *   eps = alpha sigma_1; M's eps-pseudoinverse keeps 1/(a+b), 1/(a-b) where
 *     |a +- b| > eps (Definition pseudoinverse);
 *   the residual e loses the resulting rank-2 term, written as two rank-1
 *     terms d (C0 +- C1)(R0 +- R1) with d = 1/(2 (a +- b)) or 0, C0 / C1 the
 *     residual's columns at lambda - pi / lambda, R0 its row at theta and R1
 *     that row shifted by pi (eq. lowrankRepresentationSplit).
 * Outputs (device): d [2 steps], c [2 steps][m], r [2 steps][n] in the form
 * sphere_poisson_solve_lowrank and sphere_poisson_eval_lowrank take (f is
 * approximated by sum_q d[q] c[q] r[q]); pivots [steps][2] (t, i), or NULL.
 * The loop stops once sigma_1 <= tol times the first step's sigma_1; the
 * remaining steps write d = 0, zero factors and pivots -1.  The pole
 * zero-out step of eq. ZeroOut is not applied (the grid has no pole samples).
 * work: device workspace of sphere_poisson_ge_workspace_bytes(n, m) bytes
 * (the residual and the pivot search's partials), 16-byte aligned, as is r.
 * One pivot search (one read of the grid) starts the loop; each step is then
 * three launches on hip_stream: the pivot, the factor extraction, and the
 * rank-2 update fused with the next step's pivot search (one read and one
 * write of the grid).
 * Errors: SP_ERR_INVALID_ARG (sizes, steps < 1, alpha outside [0, 1],
 * tol < 0, a NULL pointer, a small or misaligned workspace); SP_ERR_ALIAS
 * (outputs overlapping f, the workspace or each other); SP_ERR_HIP. */
size_t sphere_poisson_ge_workspace_bytes(int n_lambda, int m_theta);
int sphere_poisson_ge_lowrank(int n_lambda, int m_theta, const double* f, int steps, double alpha, double tol,
                              void* work, size_t work_bytes, double* d, double* c, double* r, int* pivots,
                              void* hip_stream);

/* For callers that cannot allocate device memory at all (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same elimination as sphere_poisson_ge_lowrank, same arguments, layout and
 * results, but with no workspace argument.  The workspace is a static device
 * array of the library, SP_GE_STATIC_BYTES (40 MiB) on every device it runs
 * on, held until the process ends; the call allocates and frees nothing (its
 * first call on a device only looks up that array's address).  Grids whose
 * workspace, sphere_poisson_ge_workspace_bytes(n, m), exceeds SP_GE_STATIC_BYTES
 * (about 5.2 million samples, e.g. 2048 x 2048 fits) give
 * SP_ERR_UNSUPPORTED_SIZE.  Every call on one device shares that array, which
 * keeps the last call's contents (each call writes every part it reads before
 * reading it): calls that overlap on one device race, so issue them on one
 * stream or serialise them.
 * Errors: as sphere_poisson_ge_lowrank, plus SP_ERR_UNSUPPORTED_SIZE and
 * SP_ERR_NO_DEVICE. */
#define SP_GE_STATIC_BYTES (40u << 20)
int sphere_poisson_ge_lowrank_static(int n_lambda, int m_theta, const double* f, int steps, double alpha, double tol,
                                     double* d, double* c, double* r, int* pivots, void* hip_stream);

/* Euclidean transpose of the linear map f -> u (integral = 0) on the grid
 * samples: fbar = S^T g.  This is the reverse-mode derivative of the solve
 * for any loss; same layout, ownership and errors as sphere_poisson_solve.
 * A MIXED adjoint applies at most one correction (its iterate is refined
 * without sin^2, whose coefficients are recovered from the transform of the
 * iterate itself): a plan with max_refine > 1 gives SP_ERR_INVALID_ARG. */
int sphere_poisson_solve_adjoint(sp_plan plan, const double* g, double* fbar,
                                 void* hip_stream, sp_info* info);

/* Heterogeneous batches (spec change 2: many right-hand sides of uneven
 * grid sizes solved by one persistent, graph-captured launch; the paper notes
 * the solver is embarrassingly parallel, Section 5).
 *
 * sphere_poisson_batch_plan builds a batch plan for `count` problems:
 * n[r], m[r]: sizes of problem r (host arrays); f[r], u[r]: device pointers
 * (host arrays of pointers), each [m[r]][n[r]] float64, bound to the plan.
 * desc: precision, max_refine (MIXED: 1..4 corrections), tol and flags
 * (SP_AUTOTUNE: measure the radix orders of every distinct size first, as
 * for sphere_poisson_plan); n_lambda, m_theta and low_k_fp64 are ignored
 * (each problem eliminates k < max(16, m/64) in float64 in MIXED).  The plan
 * allocates every problem's workspace and tables, builds the work lists
 * (one item per lambda row block or theta tile, longest first) and captures
 * the HIP graph: a counter reset kernel, then per solve stage one persistent
 * kernel per kernel build with work, each taking (problem, tile) items from
 * its list; with max_refine = R the correction stages run R times.  Every
 * problem uses integral = 0.  Every problem must fit the batch tiles (256
 * threads): n/2 up to about 4096 and m up to about 3300 (the exact bounds
 * depend on the radices), else SP_ERR_UNSUPPORTED_SIZE.
 * No u[r] may overlap another problem's f or u, nor its own f (SP_ERR_ALIAS;
 * f buffers may be shared); in SP_MIXED u[r] is scratch until the graph
 * ends, as in sphere_poisson_solve.
 * Errors: SP_ERR_INVALID_ARG (count <= 0, a NULL pointer, bad sizes or
 * precision, max_refine outside 1..4 in MIXED), SP_ERR_ALIAS,
 * SP_ERR_UNSUPPORTED_SIZE, SP_ERR_OOM, SP_ERR_HIP, SP_ERR_NO_DEVICE.
 *
 * sphere_poisson_solve_batch launches the graph once on `hip_stream`; it
 * allocates nothing.  The data is read from and written to the buffers bound
 * at planning.  `infos` may be NULL (else `count` entries, filled after a
 * synchronisation of `hip_stream`: iters, rel_correction, est_rel_err and
 * f_integral per problem, rel_residual is not computed in a batch (0)).
 * With tol > 0 a MIXED problem whose last relative correction exceeds tol
 * gets status SP_ERR_NOT_CONVERGED in its info, and the call returns that
 * code (only when infos is given: the check needs the synchronisation).
 * Calls on one batch plan must not overlap (they share its workspace and
 * counters).  Errors: SP_ERR_BAD_PLAN, SP_ERR_HIP, SP_ERR_NOT_CONVERGED.
 *
 * sphere_poisson_batch_destroy waits for the plan's last launch and releases
 * it. */
typedef struct sp_batch_s* sp_batch;
int sphere_poisson_batch_plan(sp_batch* out, int count, const int* n, const int* m, const double* const* f,
                              double* const* u, const sp_desc* desc, void* hip_stream);
int sphere_poisson_solve_batch(sp_batch batch, void* hip_stream, sp_info* infos);
int sphere_poisson_batch_destroy(sp_batch batch);

/* The info of the plan's last solve (or adjoint): synchronises `hip_stream`
 * and fills *info as SP_SYNC_INFO would have.  The norms (rel_correction,
 * rel_residual, est_rel_err) exist only when the plan has SP_SYNC_INFO or
 * SP_INFO in its flags; otherwise they read -1.  status is the last call's
 * return value, with SP_ERR_NOT_CONVERGED applied as for SP_SYNC_INFO.
 * Errors: SP_ERR_BAD_PLAN, SP_ERR_INVALID_ARG (info NULL), SP_ERR_HIP. */
int sphere_poisson_get_info(sp_plan plan, void* hip_stream, sp_info* info);

/* Diagnostic: the achievable HBM bandwidth of the device, the ceiling
 * against which the solver's kernels are read (no passage of the paper: the
 * roofline of the measurement).  kind = SP_STREAM_COPY (y[i] = x[i]),
 * SP_STREAM_READ (every element of x read once; y receives one partial sum per
 * workgroup, sphere_poisson_stream_partials(count) doubles) or SP_STREAM_WRITE
 * (y[i] = 1; x unused, may be NULL), optionally | SP_STREAM_NONTEMPORAL
 * (non-temporal loads and stores).  count: doubles; x, y device pointers,
 * 16-byte aligned; each workgroup moves one contiguous 16 KiB chunk with
 * 128-bit accesses.  Asynchronous on hip_stream; count = 0 does nothing.
 * Errors: SP_ERR_INVALID_ARG (kind, a NULL or misaligned pointer),
 * SP_ERR_ALIAS (y overlapping x), SP_ERR_UNSUPPORTED_SIZE, SP_ERR_HIP. */
#define SP_STREAM_COPY 0
#define SP_STREAM_READ 1
#define SP_STREAM_WRITE 2
#define SP_STREAM_NONTEMPORAL 0x10
size_t sphere_poisson_stream_partials(size_t count);
int sphere_poisson_stream(int kind, const double* x, double* y, size_t count, void* hip_stream);

/* Release every resource of a plan (waits for its pending work). */
int sphere_poisson_destroy(sp_plan plan);

/* Human-readable text for a status code (static storage). */
const char* sphere_poisson_strerror(int code);

/* Tangential derivatives of a grid function (Section 4, "Differentiation",
 * eq. diff_x, diff_y, diff_z): the Cartesian components of the surface
 * gradient,
 *   gx = -(sin lambda / sin theta) df/dlambda + cos lambda cos theta df/dtheta,
 *   gy =  (cos lambda / sin theta) df/dlambda + sin lambda cos theta df/dtheta,
 *   gz = -sin theta df/dtheta
 * (the z component with the chain rule's sign; the paper prints it with a
 * plus sign).  f: input, gx, gy, gz: outputs, all device [m][n] float64 on the
 * plan's grid, pairwise non-overlapping (SP_ERR_ALIAS).  The derivatives are
 * spectral (exact for band-limited f, in float64 whatever the plan's
 * precision); sin(theta) never vanishes on the half-shifted theta grid, so
 * the division is by the node values.  Asynchronous on `hip_stream`; uses the
 * plan's workspace, so calls on one plan must not overlap.
 * Errors: SP_ERR_BAD_PLAN, SP_ERR_INVALID_ARG, SP_ERR_ALIAS, SP_ERR_HIP,
 * SP_ERR_UNSUPPORTED_SIZE when two float64 rows of n/2 complex values do not
 * fit the LDS (n above about 10240). */
int sphere_poisson_tangential_gradient(sp_plan plan, const double* f, double* gx, double* gy, double* gz,
                                       void* hip_stream);

/* Vector calculus on the sphere (Section 4, Vector calculus), built on the
 * tangential derivatives above; p = (x, y, z) is the point of the unit
 * sphere and n = p its outward normal.  Vector fields are given by their
 * three Cartesian components (fx, fy, fz), each a device [m][n] float64 grid
 * function; outputs likewise.  Outputs must not overlap each other or any
 * input (SP_ERR_ALIAS).  Same precision, stream, workspace and error rules as
 * sphere_poisson_tangential_gradient.
 *   curl_scalar: (ux, uy, uz) = n x grad f            (eq. CurlScalarF)
 *   divergence:  out = d^t fx/dx + d^t fy/dy + d^t fz/dz
 *   curl:        (cx, cy, cz) = (d^t fz/dy - d^t fy/dz, d^t fx/dz - d^t fz/dx, d^t fy/dx - d^t fx/dy)
 *   vorticity:   out = n . curl(f)
 * divergence, curl and vorticity run the derivative passes once per component. */
int sphere_poisson_curl_scalar(sp_plan plan, const double* f, double* ux, double* uy, double* uz,
                               void* hip_stream);
int sphere_poisson_divergence(sp_plan plan, const double* fx, const double* fy, const double* fz, double* out,
                              void* hip_stream);
int sphere_poisson_curl(sp_plan plan, const double* fx, const double* fy, const double* fz, double* cx,
                        double* cy, double* cz, void* hip_stream);
int sphere_poisson_vorticity(sp_plan plan, const double* fx, const double* fy, const double* fz, double* out,
                             void* hip_stream);

/* Integral of a grid function over the unit sphere (Section 4,
 * "Integration", the sum2 example): 2 pi times the theta quadrature, against
 * sin(theta), of the row means, with weights exact for cosine series of
 * degree < m on the half-shifted nodes (exact for band-limited f).
 * f: input, device [m][n] float64; out: device pointer to one float64,
 * written asynchronously on `hip_stream`.  The summation order is fixed
 * (reproducible results).  Uses the plan's workspace: calls on one plan must
 * not overlap.  Errors: SP_ERR_BAD_PLAN, SP_ERR_INVALID_ARG, SP_ERR_ALIAS,
 * SP_ERR_HIP. */
int sphere_poisson_integral(sp_plan plan, const double* f, double* out, void* hip_stream);

/* Bytes of device workspace a plan for `desc` would allocate (0 on invalid desc). */
size_t sphere_poisson_workspace_bytes(const sp_desc* desc);

/* Diagnostic: the transform pipeline without the solve.  Returns, for every
 * sample, the value obtained by the forward lambda/theta transforms of
 * sin^2(theta) f followed by the inverse transforms (identity up to rounding
 * on sin^2(theta) f).  Used to test the transforms in isolation. */
int sphere_poisson_transform_roundtrip(sp_plan plan, const double* f, double* out,
                                       void* hip_stream);

/* Kernel kinds reported by the profiling calls below. */
typedef enum {
    SP_KERNEL_LAMBDA_FWD = 0,   /* lambda real DFT of a block of rows (writes the half spectrum) */
    SP_KERNEL_THETA = 1,        /* per-wavenumber theta transform + banded solve + inverse */
    SP_KERNEL_LAMBDA_INV = 2,   /* inverse lambda real DFT of a block of rows */
    SP_KERNEL_LAMBDA_MIX = 3,   /* MIXED: float32 inverse + float64 forward lambda DFT of the first iterate (kept in u) */
    SP_KERNEL_THETA_RESID = 4,  /* MIXED: float64 residual in coefficient space + float32 correction solve */
    SP_KERNEL_LAMBDA_UPD = 5,   /* MIXED: float32 inverse lambda DFT of the correction + float64 update of u */
    SP_KERNEL_REDUCE = 6,       /* norms for the convergence report */
    SP_KERNEL_LAMBDA_GRAD = 7,  /* tangential gradient: both inverse lambda DFTs of a row, combined */
    SP_KERNEL_LOWRANK = 8,      /* low-rank right-hand side: rank-K product into the half spectrum */
    SP_KERNEL_EVAL_COEFFS = 9,  /* pointwise evaluation: cosine / sine coefficients of the theta factors */
    SP_KERNEL_EVAL = 10,        /* pointwise evaluation: Horner sums at the points */
    SP_KERNEL_KINDS = 11
} sp_kernel_kind;

/* Diagnostic profiling: with `capacity` > 0 every later kernel launch of this
 * plan is bracketed by HIP events recorded on the launch stream, until
 * `capacity` launches have been recorded (0 disables and frees the events).
 * Errors: SP_ERR_BAD_PLAN, SP_ERR_INVALID_ARG (capacity < 0), SP_ERR_HIP. */
int sphere_poisson_profile_enable(sp_plan plan, int capacity);

/* Waits for the recorded launches and returns, per sp_kernel_kind, the summed
 * duration in milliseconds (total_ms[SP_KERNEL_KINDS]) and the launch count
 * (counts[SP_KERNEL_KINDS]); then clears the record.  Either array may be NULL. */
int sphere_poisson_profile_read(sp_plan plan, double* total_ms, int* counts);

#ifdef __cplusplus
}
#endif

#endif /* SPHERE_POISSON_H */
