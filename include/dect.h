/*
 * dect.h -- C-ABI of the MI355X (gfx950) library for one-step iterative
 * estimation of effective atomic number Z and relative electron density rho_e
 * from dual-energy fan-beam sinograms.
 *
 * Method: Wang et al., "One-step Iterative Estimation of Effective Atomic
 * Number and Electron Density for Dual Energy CT" (arXiv 2308.01290):
 * objective (10) with its gradient-L0 regularisers on f1, f2, rho_e and Z^m,
 * split by half-quadratic splitting into subproblems (13a)-(13d) and iterated
 * as Algorithm 1.  Here the two image-domain data terms of (10) are replaced by
 * projection-domain terms eta*||A(f1 mu1(E_k) + f2 mu2(E_k)) - p_k||^2, A the
 * fan-beam projector and p_k the post-log sinograms, so every iteration runs a
 * forward projection and a matched back-projection of both energy channels.
 *
 * Conventions shared by every entry point
 *   - Array pointers are DEVICE pointers (hipMalloc / torch CUDA tensors) owned
 *     by the caller; the library never frees them.  Host pointers are marked.
 *   - Images are float32 [batch][n_y][n_x], sinograms float32
 *     [batch][n_views][n_det], row-major and contiguous.  Image row i, column k
 *     is the half-open square [x0 + k*d, x0 + (k+1)*d) x [y0 + i*d, y0 + (i+1)*d)
 *     with x0 = -n_x*d/2, y0 = -n_y*d/2 (mm), d = pixel_mm.
 *   - Sinogram values are post-log line integrals p = -ln(I/I0) (dimensionless);
 *     attenuation images are in 1/mm; system-matrix entries in mm.
 *   - Calls validate their arguments on the host and return a negative status
 *     before anything is enqueued; otherwise they only ENQUEUE work on `stream`
 *     and return DECT_OK.  Results are valid after the caller synchronises the
 *     stream.  Asynchronous device faults surface at that synchronisation.
 *   - dect_last_error() returns a thread-local message for the last failure.
 *   - No exception crosses the ABI.  Calls are reentrant given distinct
 *     workspaces / solver handles; one handle must not be used from two host
 *     threads at once.
 */
#ifndef DECT_H
#define DECT_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    DECT_OK = 0,
    DECT_EINVAL = -1,       /* invalid argument or geometry                 */
    DECT_EWORKSPACE = -2,   /* caller workspace too small or misaligned     */
    DECT_ENOMEM = -3,       /* device allocation failed                     */
    DECT_EDEVICE = -4,      /* a HIP runtime call failed                    */
    DECT_EUNSUPPORTED = -5, /* valid request the library does not implement */
    DECT_EBUSY = -6         /* no free slot (dect_engine_admit)             */
};

/* Fan-beam geometry (mm, radians).
 * View v has angle theta_v = angle0_rad + v*arc_rad/n_views; the source sits at
 * sid_mm*(cos, sin) theta_v; the flat detector is centred at
 * -(sdd_mm - sid_mm)*(cos, sin) theta_v with axis e = (-sin, cos) theta_v, and
 * bin j is centred at u_j = (j - (n_det-1)/2)*det_pitch_mm + det_offset_mm
 * along e.  Ray (v, j) is the line from the source to that bin centre.
 * det_pitch_mm = 0 selects the pitch whose fan just covers the image corners:
 * 2*sdd*tan(asin(R/sid))/n_det, R = pixel_mm*hypot(n_x, n_y)/2.
 * Valid geometry: all sizes >= 1, pixel_mm > 0, sdd_mm > sid_mm > 0, and the
 * image half-diagonal R < sid_mm and R < sdd_mm - sid_mm. */
typedef struct dect_geometry {
    int32_t n_x, n_y;
    double pixel_mm;
    int32_t n_views;
    double angle0_rad, arc_rad;
    int32_t n_det;
    double det_pitch_mm, det_offset_mm;
    double sid_mm, sdd_mm;
} dect_geometry;

/* Method parameters.  Zero in the marked fields selects the default.
 *   E_lo_keV, E_hi_keV   effective acquisition energies (60, 90)
 *   E1_keV, E2_keV       synthesis energies of eq. (2a,b) (50, 200)
 *   m, n, Cp             photoelectric model rho_e*Cp*Z^m/E^n, Section II-B
 *                        (3.94, 3.2, 9.8e-24); the coefficient is normalised
 *                        to water, Cp*Z_w^(3.8 - m), so water keeps the
 *                        printed m = 3.8 value
 *   Z_w                  effective atomic number of water (7.42)
 *   basis_Z, basis_rho   the two basis materials of eq. (1a,b)
 *                        (SB3 cortical bone 14.14/1.69, water 7.42/1.00)
 *   lambda               gradient-L0 weight of eq. (5)/(10) (0.01)
 *   beta0, beta_max      relaxation schedule of Algorithm 1 (0 -> 2*lambda, 1e5)
 *   kappa                beta growth rate (0 -> (beta_max/beta0)^(1/n_iter))
 *   eta, xi              projection-data and coupling weights (0 -> the
 *                        normalisations that give water unit curvature)
 *   n_iter               outer iterations K of Algorithm 1 (>= 1)
 *   f_inner              steepest-descent/CG steps on the f-subproblem per
 *                        outer iteration (this library: 1)
 *   t_tol, t_maxit       PCG tolerance (relative residual) and cap of the
 *                        Z^m subproblem (1e-7, 200); Z = Zw*t'^(1/m) is
 *                        ill-conditioned where t' is small, which is what
 *                        sets this tolerance
 *   rho_min, t_min       output mask: Z = 0 where rho_e < rho_min; t' clamp
 *                        (0.1, 1e-6)
 *   t_precond            preconditioner of the Z^m PCG, a DECT_PRECOND_*
 *                        value (DECT_PRECOND_AUTO: the multigrid V-cycle
 *                        where the image sizes admit it, else Jacobi below
 *                        beta = 1.5 and the scaled FFT inverse above).  The
 *                        choice changes the iterate only within t_tol.
 *   storage              precision of stored iterates, a DECT_STORAGE_* value
 *                        (sinogram form only; the image-domain form returns
 *                        DECT_EUNSUPPORTED for anything but FP32). */
typedef struct dect_params {
    double E_lo_keV, E_hi_keV, E1_keV, E2_keV;
    double m, n, Cp, Z_w;
    double basis_Z[2], basis_rho[2];
    double lambda, beta0, beta_max, kappa;
    double eta, xi;
    int32_t n_iter, f_inner;
    double t_tol;
    int32_t t_maxit;
    double rho_min, t_min;
    int32_t t_precond;
    int32_t storage;
} dect_params;

/* Values of dect_params.storage.  Arithmetic is FP32 (FP64 where stated) in
 * every mode; only what is stored between kernels changes.
 *   DECT_STORAGE_FP32        everything in FP32 (default)
 *   DECT_STORAGE_BF16        the projector operands in BF16, rounded to
 *                            nearest even when written: the search direction
 *                            the forward projector reads, the residual
 *                            sinograms the back-projector reads, and the
 *                            line-search sinograms; ray sums and
 *                            back-projection accumulate in FP32, the line
 *                            search uses the stored direction
 *   DECT_STORAGE_BF16_STATE  as BF16, and the state images f1, f2, rho_e, t'
 *                            rounded to BF16 after every write (start and
 *                            each outer iteration); the residual sinograms
 *                            are updated incrementally as in FP32 mode, so
 *                            they carry the projection of the f rounding */
enum {
    DECT_STORAGE_FP32 = 0,
    DECT_STORAGE_BF16 = 1,
    DECT_STORAGE_BF16_STATE = 2
};

/* Values of dect_params.t_precond.  DECT_PRECOND_MULTIGRID needs every image
 * side above 64 to be a multiple of 16 down to 64 (sides halve per level) and
 * a coarsest grid (first odd side, or 1 x 1) of at most 64 pixels; otherwise
 * the solver returns DECT_EUNSUPPORTED. */
enum {
    DECT_PRECOND_AUTO = 0,
    DECT_PRECOND_JACOBI = 1,
    DECT_PRECOND_FFT = 2,
    DECT_PRECOND_MULTIGRID = 3
};

/* Fill *p with the defaults listed above (HOST pointer). */
void dect_default_params(dect_params* p);

/* Validate *g (HOST pointer) and replace det_pitch_mm = 0 by the
 * corner-covering pitch.  Returns DECT_OK or DECT_EINVAL. */
int dect_resolve_geometry(dect_geometry* g);

/* Linear attenuation (1/mm) at E_lo and E_hi of n materials with given
 * (Z, rho_e), from the model of Section II-B (eq. (3a,b) scaled by the
 * electron density of water).  HOST pointers, FP64.  Used to synthesise
 * inputs; not part of the solve. */
int dect_attenuation(const dect_params* p, const double* Z, const double* rho_e, int64_t n,
                     double* mu_lo, double* mu_hi);

/* Forward projection sino = A img: for every ray, the sum of pixel values
 * times the ray's chord length through each pixel square (exact, Siddon-type
 * traversal, FP32 with compensated ray sums).  img [batch][n_y][n_x] ->
 * sino [batch][n_views][n_det].  Needs a device-side table the library keeps
 * per geometry (allocated on first use).  A square image (n_x = n_y, a
 * multiple of 32) with a full turn of views (arc 2*pi, n_views a multiple of
 * 4) is closed under quarter turns of the scanner: the table then holds a
 * quarter of the views and each ray's traversal serves four rays; with
 * angle0 = 0 and det_offset = 0 the image diagonal is a further mirror and
 * the back-projector evaluates each chord once for eight rays.  The chord
 * lengths are those of the same rays, so results agree with the general
 * traversal within FP32 rounding. */
int dect_project(const dect_geometry* g, const float* img, float* sino, int32_t batch,
                 hipStream_t stream);

/* Back-projection img = A^T sino with the same chord lengths as dect_project
 * (the exact adjoint up to FP32 rounding; voxel-driven gather, deterministic). */
int dect_backproject(const dect_geometry* g, const float* sino, float* img, int32_t batch,
                     hipStream_t stream);

/* Flat-detector fan-beam filtered back-projection (cosine weighting, Ram-Lak
 * filter, distance-weighted back-projection with linear interpolation): the
 * attenuation images that Algorithm 1 requires as input, reconstructed from
 * the sinograms.  sino [batch][n_views][n_det] -> img [batch][n_y][n_x]. */
int dect_fbp(const dect_geometry* g, const float* sino, float* img, int32_t batch,
             hipStream_t stream);

/* One half-quadratic-splitting step of the gradient-L0 model, eq. (5)-(9):
 *   (h, v) = hard threshold (9) of the periodic forward differences of g^(k)
 *            ((h, v) = 0 where dx^2 + dy^2 <= lambda/beta, evaluated in FP32:
 *            a pixel within rounding of the threshold may go either way);
 *   g^(k+1) = argmin ||w*g - g_tilde||^2 + beta*||D g - (h, v)||^2,
 * i.e. (diag(w^2) + beta D^T D) g = w*g_tilde + beta D^T (h, v), periodic.
 * weight == NULL means w = 1 and uses the FFT closed form of Section II-C;
 * otherwise preconditioned CG to relative residual `tol` (at most `max_iter`
 * iterations).  g is in/out ([batch][n_y][n_x]); h_out, v_out may be NULL.
 * ws/ws_bytes: device workspace of at least dect_l0_step_workspace_bytes()
 * bytes, 256-byte aligned; NULL lets the library allocate it (stream-ordered).
 * Sizes: n_x, n_y of the form 2^a*3^b with b <= 1, 8 <= n <= 1024. */
size_t dect_l0_step_workspace_bytes(int32_t n_y, int32_t n_x, int32_t batch, int weighted);
int dect_l0_step(const float* g_tilde, const float* weight, float* g, float* h_out, float* v_out,
                 int32_t n_y, int32_t n_x, int32_t batch, double lambda, double beta,
                 double tol, int32_t max_iter, void* ws, size_t ws_bytes, hipStream_t stream);

/* Allocation-free variant of dect_l0_step with unit weight (the FFT closed
 * form), for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  It
 * allocates nothing: its complex scratch is a static device array in the
 * library, one per GPU (held until the process ends), of
 * dect_l0_step_static_max_values() float2 values (2^21, 16 MiB); batch*n_y*n_x
 * above that returns DECT_EINVAL before anything is enqueued.  Every call on a
 * GPU shares that array, so calls that overlap on one GPU (other streams or
 * threads) race; calls ordered on one stream do not.  Arguments, layout,
 * results and other errors are those of dect_l0_step with weight = NULL; the
 * results equal dect_l0_step's bit for bit (same kernels, same order). */
size_t dect_l0_step_static_max_values(void);
int dect_l0_step_static(const float* g_tilde, float* g, float* h_out, float* v_out, int32_t n_y,
                        int32_t n_x, int32_t batch, double lambda, double beta, hipStream_t stream);

/* ---- solver -------------------------------------------------------------
 * A solver holds one batch of slices that share parameters and the image grid
 * (n_x, n_y, pixel_mm), and all per-iteration state on the device: basis
 * images f1, f2, rho_e, the
 * normalised t' = Z^m/Z_w^m, the combined residual sinograms and scratch.
 * Algorithm 1, sinogram form, per outer iteration k (all updates read iterate k):
 *   f-step   one steepest-descent step with exact line search on the
 *            f-subproblem (13a) with projection data terms (one back-projection
 *            of the residuals, one forward projection of the direction);
 *   rho step subproblem (13b) by the FFT closed form;
 *   t' step  subproblem (13c) by preconditioned CG;
 *   beta <- kappa*beta.
 * Initialisation: FBP of both sinograms, then the per-pixel closed forms of
 * Algorithm 1's initialisation. */
typedef struct dect_solver dect_solver;

/* Workspace bytes a solver needs for this geometry/params/batch. */
size_t dect_solve_workspace_bytes(const dect_geometry* g, const dect_params* p, int32_t batch);

/* Create a solver bound to `stream`.  ws == NULL: the library allocates the
 * workspace; otherwise the caller's device buffer of >= the size above (256-
 * byte aligned) is used and must outlive the solver.  *out is a HOST handle. */
int dect_solver_create(const dect_geometry* g, const dect_params* p, int32_t batch, void* ws,
                       size_t ws_bytes, hipStream_t stream, dect_solver** out);

/* Batches of uneven slices: geoms is a HOST array of `batch` geometries that
 * share n_x, n_y and pixel_mm; views, bins, detector and distances may
 * differ per slice (DECT_EINVAL otherwise).  Every launch of an iteration
 * covers all slices.  The sinogram arguments of dect_solver_init /
 * set_state are then the slices' sinograms back to back: slice z starts at
 * element sum over z' < z of n_views(z') * n_det(z').  Images stay
 * [batch][n_y][n_x].  Each slice follows the iteration it follows alone: its
 * own data weight eta (from its geometry unless set), its own line search and
 * PCG stopping test; beta schedule and parameters are shared. */
size_t dect_solve_workspace_bytes_multi(const dect_geometry* geoms, const dect_params* p,
                                        int32_t batch);
int dect_solver_create_multi(const dect_geometry* geoms, const dect_params* p, int32_t batch,
                             void* ws, size_t ws_bytes, hipStream_t stream, dect_solver** out);
int dect_solver_destroy(dect_solver* s);

/* Initialise from the sinograms (FBP + closed forms); k = 0. */
int dect_solver_init(dect_solver* s, const float* sino_lo, const float* sino_hi);

/* Load an explicit state (f1, f2, rho_e, t' images) at outer iteration k
 * together with the sinograms it is fitted to. */
int dect_solver_set_state(dect_solver* s, const float* sino_lo, const float* sino_hi,
                          const float* f1, const float* f2, const float* rho, const float* t,
                          int32_t k);

/* Run n outer iterations (k -> k + n). */
int dect_solver_iterate(dect_solver* s, int32_t n);

/* Copy the state images out (any pointer may be NULL). */
int dect_solver_get_state(const dect_solver* s, float* f1, float* f2, float* rho, float* t);

/* Output maps: rho_e, and Z = Z_w*max(t', t_min)^(1/m) with Z = 0 where
 * rho_e < rho_min. */
int dect_solver_finish(dect_solver* s, float* Z, float* rho_e);

/* Number of outer iterations done and the PCG iterations spent in the last
 * t' step (HOST query; synchronises the solver's stream). */
int dect_solver_stats(const dect_solver* s, int32_t* k, int32_t* last_pcg_iters);

/* Launch schedule of a solver's outer iterations.  Every choice changes only
 * how the work is mapped onto the device, never an operation or its
 * summation order, so results are bit-identical under every schedule.
 *   fp_rays_per_lane  line-search forward projection of square quarter-turn
 *                     symmetric slices: 4 = each lane steps one table ray
 *                     and sums its four turned rays; 1 = one ray per lane
 *                     (the kernel of the general case).  Slices of neither
 *                     symmetry always take 1, in a launch of their own when
 *                     the batch mixes the two kinds.
 *   bp_cu_percent     workgroups of the symmetric back-projectors as a
 *                     percentage of the CUs (0 = automatic: half the CUs up
 *                     to one tile orbit per CU, all CUs beyond; else 10..400)
 *   rho_stream        1 = the rho_e step of the sinogram form on a stream of
 *                     its own, 0 = on the f-step's stream
 *   graphs            1 = the t' PCG's first chunk per outer iteration
 *                     replayed from a HIP graph (see dect_solver_set_graphs)
 *   pcg_chunk_extra   PCG iterations enqueued in the first chunk beyond the
 *                     previous outer iteration's count (0..8); the device
 *                     stopping test makes extra iterations free of effect
 *   pcg_chunk_first   order in which the host enqueues an outer iteration
 *                     once the previous one's back-projection is queued:
 *                     1 = the PCG's first chunk, then the f-step and rho_e
 *                     work; 0 = the PCG's set-up, then the f-step and rho_e
 *                     work, then the chunk (the f-step's kernels then need not
 *                     wait for the host to enqueue the chunk)
 * A new solver starts with {4, 0, 1, 0, 0, 1}. */
typedef struct dect_schedule {
    int32_t fp_rays_per_lane;
    int32_t bp_cu_percent;
    int32_t rho_stream;
    int32_t graphs;
    int32_t pcg_chunk_extra;
    int32_t pcg_chunk_first;
} dect_schedule;

/* Read or replace the schedule (DECT_EINVAL for a NULL argument or a value
 * outside the ranges above; set takes effect at the next iterate call). */
int dect_solver_get_schedule(const dect_solver* s, dect_schedule* out);
int dect_solver_set_schedule(dect_solver* s, const dect_schedule* in);

/* Autotuner: times `iters` outer iterations from dect_solver_init (or
 * dect_image_solver_init for an image-domain solver) on the given inputs,
 * `reps` times per candidate schedule (median), over the knobs above one at
 * a time (coordinate descent from the current schedule; a change is kept
 * when it is at least 2% faster), and leaves the fastest schedule set.
 * Timing is by HIP events on the solver's stream around each trial's
 * iterations.  sino_lo/sino_hi: DEVICE pointers as for dect_solver_init (the
 * attenuation images for an image-domain solver).  chosen and ms_per_iter
 * (the chosen schedule's median time per outer iteration) may be NULL.  The
 * solver's iterate is left at the last trial's: call dect_solver_init (or
 * set_state) before solving.  iters in 1..100, reps in 1..20. */
int dect_solver_autotune(dect_solver* s, const float* sino_lo, const float* sino_hi,
                         int32_t iters, int32_t reps, dect_schedule* chosen,
                         double* ms_per_iter);

/* Graph replay of the t' PCG's launch-bound inner loop: with enable != 0,
 * the first chunk of PCG iterations of every outer iteration (the multigrid
 * V-cycles with the fused update, about five small kernels per PCG
 * iteration) is captured once per chunk length and pair of t' buffers as a
 * HIP graph and replayed with one hipGraphLaunch.  Applies when the
 * multigrid PCG is in use and the solver has its own streams (a caller
 * stream that is the legacy NULL stream still gets them); otherwise the
 * iterations are launched one by one as before.  The replayed launches are
 * those of the eager path, so results are bit-identical.  The solver keeps at
 * most 16 instantiated graphs (dropped, after a stream synchronisation, when
 * the cache is full, when graphs are disabled, and by dect_solver_destroy).
 * Same as setting dect_schedule.graphs.  Returns DECT_EINVAL for a NULL
 * solver. */
int dect_solver_set_graphs(dect_solver* s, int enable);

/* Optional timing of the two system-matrix kernels: with bit 0 of `enable`
 * set, the solver records HIP events on its stream around every
 * back-projection and forward projection launch of the outer iterations
 * (with bit 2 also set, around the back-projections only, which halves the
 * events in the iteration); bit 1 records the iteration timeline
 * (dect_solver_timeline).  dect_solver_timing synchronises
 * the stream, returns the summed durations (ms) and launch counts since the
 * last call, and resets them.  Any output pointer may be NULL.  For an
 * image-domain solver the first pair times each iteration's f-step (the
 * joint FFT solve, one interval per iteration) and the second stays zero. */
int dect_solver_enable_timing(dect_solver* s, int enable);
int dect_solver_timing(dect_solver* s, double* backproject_ms, int32_t* backproject_launches,
                       double* project_ms, int32_t* project_launches);

/* Iteration timeline of the sinogram form, recorded while bit 1 of the timing
 * switch is set (HIP events on the solver's streams, at most 4096 outer
 * iterations between
 * two reads): for every outer iteration that follows another of the same
 * solve, five times in microseconds after the previous iteration's update of
 * f, in this order:
 *   0  the f-step's stream reaches the gradient (its back-projection done and
 *      t'^(k) available), 1  its forward projection done, 2  its update done
 *      (the iteration period), 3  the t' PCG's set-up done, 4  the PCG done
 *      (its last chunk's stopping flags copied).
 * Writes at most max_rows rows of five floats to out_us (host memory), the
 * row count to *rows, and clears the record.  Waits for the recorded events.
 * Returns DECT_EINVAL for a NULL solver or output; an image-domain solver
 * records nothing (*rows = 0). */
int dect_solver_timeline(dect_solver* s, float* out_us, int32_t max_rows, int32_t* rows);

/* Whole solve: create, init, n_iter iterations, finish, destroy. */
int dect_solve(const float* sino_lo, const float* sino_hi, const dect_geometry* g,
               const dect_params* p, float* Z_out, float* rho_out, int32_t batch, void* ws,
               size_t ws_bytes, hipStream_t stream);
/* The same for a batch of uneven slices (see dect_solver_create_multi). */
int dect_solve_multi(const float* sino_lo, const float* sino_hi, const dect_geometry* geoms,
                     const dect_params* p, float* Z_out, float* rho_out, int32_t batch, void* ws,
                     size_t ws_bytes, hipStream_t stream);

/* ---- batches of mixed image sizes ------------------------------------------
 * One handle for a batch of slices whose image grids differ too (n_x, n_y,
 * pixel_mm), as in a batch of 256^2, 384^2 and 512^2 slices.  Slices of one
 * image grid form a group that runs as one uneven batch (every launch of an
 * iteration covers the whole group, see dect_solver_create_multi); an
 * iteration enqueues the work of every group before it waits for any group's
 * PCG stopping flags, so the groups overlap on the device.  Every slice's
 * result equals its solve alone (dect_solve of that slice), bit for bit.
 * Sinograms: slices back to back in the order of geoms (slice z starts at
 * element sum_{z'<z} n_views(z') n_det(z')); images likewise (slice z at
 * element sum_{z'<z} n_x(z') n_y(z')).  All DEVICE, caller-owned; init reads
 * the sinograms during its enqueued work only.  The library allocates each
 * group's workspace (stream-ordered on `stream`).  Errors as for the solver
 * calls; parameters are shared (n_iter is used by dect_solve_uneven only). */
typedef struct dect_uneven dect_uneven;
int dect_uneven_create(const dect_geometry* geoms, int32_t batch, const dect_params* p,
                       hipStream_t stream, dect_uneven** out);
int dect_uneven_destroy(dect_uneven* u);
/* Number of image-grid groups (HOST pointer). */
int dect_uneven_groups(const dect_uneven* u, int32_t* n_groups);
int dect_uneven_init(dect_uneven* u, const float* sino_lo, const float* sino_hi);
int dect_uneven_iterate(dect_uneven* u, int32_t n);
int dect_uneven_finish(dect_uneven* u, float* Z_out, float* rho_out);
/* dect_solver_autotune on each group alone (iters, reps as there; the inputs
 * as for dect_uneven_init); then, one group at a time, a group's choice is
 * kept only if the whole handle (its groups' iterations interleaved) runs at
 * least 2% faster with it than without.  The handle's iterate is left at the
 * last trial's: init before solving. */
int dect_uneven_autotune(dect_uneven* u, const float* sino_lo, const float* sino_hi, int32_t iters,
                         int32_t reps);
int dect_uneven_get_schedule(const dect_uneven* u, int32_t group, dect_schedule* out);
/* Whole solve of such a batch: create, init, n_iter iterations, finish, destroy. */
int dect_solve_uneven(const float* sino_lo, const float* sino_hi, const dect_geometry* geoms,
                      const dect_params* p, float* Z_out, float* rho_out, int32_t batch,
                      hipStream_t stream);

/* ---- image-domain form ----------------------------------------------------
 * Algorithm 1 on attenuation images instead of sinograms: the data terms of
 * objective (10) are eta_i*||C_k1 f1 + C_k2 f2 - mu_k||^2 for the two
 * acquisition energies, and the f-subproblem (13a) is solved for (f1, f2)
 * jointly, which satisfies both printed FFT closed forms at once: per
 * frequency the 2x2 system
 *   (H + beta |F D|^2 I) F(f) = F(b) + beta F(D^T HT(D f^(k))),
 *   H = eta_i C^T C + xi Ms^T Ms,  b_i = eta_i sum_k C_ki mu_k + xi sum_j Ms_ji T_j.
 * (The printed forms taken one basis at a time, each with the other at
 * iterate k, do not converge at low frequencies once the coupling target
 * lags; (13a) asks for the joint minimiser.)
 * The rho_e and t' steps, the beta schedule, the initialisation (the per-pixel
 * closed forms) and the output are those of the sinogram form.  eta = 0 in
 * dect_params selects eta_i = 1 / (mu_w(E_lo)^2 + mu_w(E_hi)^2), water's
 * unit curvature in f2.
 * Inputs mu_lo, mu_hi: [batch][n_y][n_x] attenuation images (1/mm, DEVICE),
 * copied into the workspace by init / set_state (the caller's buffers are
 * free once that enqueued work has run).  n_x, n_y as for dect_l0_step.  The
 * handle is a dect_solver: dect_solver_iterate, _get_state, _finish, _stats
 * and _destroy apply to it; dect_solver_init and _set_state reject it (and
 * the two calls below reject a sinogram solver) with DECT_EINVAL. */
size_t dect_image_workspace_bytes(int32_t n_x, int32_t n_y, const dect_params* p, int32_t batch);
int dect_image_solver_create(int32_t n_x, int32_t n_y, const dect_params* p, int32_t batch,
                             void* ws, size_t ws_bytes, hipStream_t stream, dect_solver** out);
/* Initialise from the attenuation images (closed forms); k = 0. */
int dect_image_solver_init(dect_solver* s, const float* mu_lo, const float* mu_hi);
/* Load an explicit state at outer iteration k with the images it is fitted to. */
int dect_image_solver_set_state(dect_solver* s, const float* mu_lo, const float* mu_hi,
                                const float* f1, const float* f2, const float* rho, const float* t,
                                int32_t k);
/* Whole solve: create, init, n_iter iterations, finish, destroy. */
int dect_solve_image(const float* mu_lo, const float* mu_hi, int32_t n_x, int32_t n_y,
                     const dect_params* p, float* Z_out, float* rho_out, int32_t batch, void* ws,
                     size_t ws_bytes, hipStream_t stream);

/* ---- continuous batching ------------------------------------------------
 * An engine is a pool of `slots` slots on one image grid (n_x, n_y, pixel_mm)
 * for serving single-slice requests as they arrive.  Each slot holds one
 * request at its own outer iteration: its own fan geometry (at most
 * max_views x max_det), data weight eta, iteration budget n_iter and beta
 * schedule (beta0 -> beta_max over n_iter iterations; params->kappa must be
 * 0).  A step advances every occupied slot by one iteration of Algorithm 1
 * (sinogram form) in the same launches; a slot that completes its budget
 * enqueues its Z and rho_e maps into the caller's buffers and becomes free.
 * A request's result is the same as dect_solve of that slice alone (bit for
 * bit).  All calls enqueue on the engine's stream; outputs are valid after
 * the caller synchronises it. */
typedef struct dect_engine dect_engine;
size_t dect_engine_workspace_bytes(int32_t n_x, int32_t n_y, double pixel_mm, int32_t slots,
                                   int32_t max_views, int32_t max_det, const dect_params* p);
int dect_engine_create(int32_t n_x, int32_t n_y, double pixel_mm, int32_t slots,
                       int32_t max_views, int32_t max_det, const dect_params* p, void* ws,
                       size_t ws_bytes, hipStream_t stream, dect_engine** out);
int dect_engine_destroy(dect_engine* e);
/* Admit a request (sinograms [n_views][n_det], DEVICE, read during this call's
 * enqueued work only; Z_out / rho_out [n_y][n_x] DEVICE, written when the
 * request completes).  DECT_EBUSY when every slot is occupied; *slot_out
 * (HOST, nullable) receives the slot. */
int dect_engine_admit(dect_engine* e, const dect_geometry* g, const float* sino_lo,
                      const float* sino_hi, int32_t n_iter, float* Z_out, float* rho_out,
                      int32_t* slot_out);
/* One outer iteration of every occupied slot. */
int dect_engine_step(dect_engine* e);
/* Up to n outer iterations of every occupied slot, pipelined across the
 * iterations like dect_solver_iterate, and no more than the first slot to
 * complete still needs (so that its slot can be refilled after the call).
 * The results equal those of as many dect_engine_step calls.  *done_iters
 * (HOST, nullable) receives the number run (0 with no occupied slot).
 * DECT_EINVAL for a NULL engine or n < 1. */
int dect_engine_step_n(dect_engine* e, int32_t n, int32_t* done_iters);
/* Cancel the request in `slot` between steps: the slot is freed at once
 * (admittable again), the request's outputs are never written and it is not
 * reported by dect_engine_completed.  The other slots' results are unchanged
 * (each slot follows its own iteration).  DECT_EINVAL when the slot holds no
 * request. */
int dect_engine_cancel(dect_engine* e, int32_t slot);
/* Occupied and free slots (HOST pointers, nullable). */
int dect_engine_status(const dect_engine* e, int32_t* active, int32_t* free_slots);
/* Slots completed since the last call, oldest first (HOST array of cap). */
int dect_engine_completed(dect_engine* e, int32_t* slots, int32_t cap, int32_t* n);

const char* dect_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DECT_H */
