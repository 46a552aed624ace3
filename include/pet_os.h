/*
 * pet_os.h -- C ABI of the MI355X ordered-subsets PET reconstruction library.
 *
 * Implements SDP-BSREM (Guo et al., "A Fast Convergent Ordered-Subsets
 * Algorithm with Subiteration-Dependent Preconditioners for PET Image
 * Reconstruction", arXiv 2111.07886): minimise
 *     Phi(f) = <Af,1> - <ln(Af+gamma), g> + beta R(f)          (eq:ObjectiveFunction)
 * with the relative difference prior R (eq:RDP) over the box
 * B = {0 <= f_j <= U} (eq:BoundedSet) by the iteration of Table I
 * (tab:SDPBSREM):
 *     f~ = f - lambda_k diag(alpha_{k,i} nu^{k,i}) S(f) grad Phi_i(f),   f <- P_t(f~)
 * with S from eq:preconditioner/eq:pj, P_t from eq:OperatorPt, lambda_k =
 * lambda0/(a k + 1), alpha_{k,i} from preconditioner:Nesterov (M1, P1) or
 * preconditioner:KM (M2, P2) and nu^{k,i} from eq:nuki (P1, P2).
 *
 * Notation: the paper's g (counts), gamma (background mean) and f (image) are
 * the arguments y, r and f below.
 *
 * Conventions shared by every call
 *   - Images are FP32, contiguous [nz][ny][nx] (x fastest); nz = 1 in 2D.
 *     Pixel centres at ((i - (n-1)/2) * v); cells are half-open.
 *   - Sinograms are FP32, contiguous [plane][angle][bin] (bins fastest); one
 *     plane in 2D.  Angle a is theta_a = a*pi/n_angles; bin b sits at
 *     s_b = (b - (n_radial-1)/2) * ds; ray (a,b) is x cos + y sin = s_b.
 *     3D: rings at slice centres (n_rings == nz, ring_pitch == vz); the LOR of
 *     rings (r1, r2) climbs linearly from z_r1 to z_r2 between the two points
 *     where the transaxial line meets the detector circle of radius
 *     det_radius; span-1 plane order is ring difference d = 0,+1,-1,...,+D,-D
 *     with ascending r1 inside each d.
 *   - Subset i (1..M) is every angle a with a mod M == i-1 (interleaved).
 *   - Pointers named f, y, r, q, w, out are DEVICE pointers owned by the
 *     caller (e.g. torch tensors); they must stay valid until the work queued
 *     on `stream` has finished.  `stream` is a hipStream_t (NULL: default).
 *   - Handles (pet_os_geom, pet_os_state) are owned by the library.
 *   - Every call returns PET_OS_OK (0) or a negative PET_OS_ERR_* code and sets
 *     a thread-local message readable with pet_os_last_error().  Arguments are
 *     validated before anything is queued: a failing call changes nothing.
 *   - Data check (the problem statement of Sec. II-A and eq:BoundedSet): the
 *     reconstruction entry points (pet_os_subiteration, pet_os_run,
 *     pet_os_reconstruct, pet_os_batch_add, served admission) reject with
 *     PET_OS_ERR_INVALID_ARG data in which a count y is negative or not
 *     finite, a background value r is not > 0 or not finite (gamma in
 *     R^p_{++}), or an image value f lies outside [0, U] or is not finite
 *     (OSEM: f >= 0); with P1/P2 and J0 = 0 f must also have a positive
 *     entry (its mean divides the gradient magnitude of mu).  The check is
 *     one device pass over y, r and f followed by a synchronisation of
 *     `stream`; a state makes it when it first sees a (f, y, r) triple of
 *     buffers, not again while the same buffers come back.
 *   - A 3D state (up to 64 rings and 15 ring differences) also copies y and r
 *     into a bin-major layout of its own (8 bytes per bin, allocated at the
 *     first subiteration) when it first sees a (y, r) pair of buffers, and
 *     reads the copy while the same pair comes back: new contents in the
 *     same buffers need a state of their own.  If that allocation fails, or
 *     for pet_os_reconstruct_noalloc, y and r are read where they are.
 *   - Calls are asynchronous on `stream` unless stated otherwise.
 */
#ifndef PET_OS_H
#define PET_OS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PET_OS_OK 0
#define PET_OS_ERR_INVALID_ARG (-1)
#define PET_OS_ERR_OUT_OF_MEMORY (-2)
#define PET_OS_ERR_DEVICE (-3)
#define PET_OS_ERR_BUDGET (-4)
#define PET_OS_ERR_NUMERIC (-5)
#define PET_OS_ERR_TIMEOUT (-6)
#define PET_OS_ERR_STATE_MISMATCH (-7)

/* preconditioner variants of Sec. III-B: BSREM (alpha = nu = 1), M1/P1
 * (Nesterov alpha), M2/P2 (KM alpha); P* also use the smoothness vector nu.
 * PET_OS_OSEM: the ordered-subsets EM of Hudson and Larkin, used by the
 * paper (Sec. IV-C) to initialise SDP-BSREM:
 *   f_j <- f_j (A_i^T (y_i / (A_i f + r_i)))_j / (A_i^T 1)_j,
 * f_j kept where the subset sensitivity (A_i^T 1)_j is 0.  It uses no
 * penalty, relaxation or clamp; of the parameters only beta, gamma_R and
 * eps (objective evaluations) and objective_every are read.  States and
 * pet_os_reconstruct only (not the batched or served paths); the state
 * holds the M subset sensitivities (M * n_voxels floats). */
#define PET_OS_BSREM 0
#define PET_OS_M1 1
#define PET_OS_M2 2
#define PET_OS_P1 3
#define PET_OS_P2 4
#define PET_OS_OSEM 5

typedef struct pet_os_geom pet_os_geom;
typedef struct pet_os_state pet_os_state;
typedef void* pet_os_stream; /* hipStream_t */

/* Scanner / image geometry (system model of Sec. IV-A, one line per bin). */
typedef struct {
    int32_t dim;              /* 2 or 3 */
    int32_t nx, ny, nz;       /* image size; nz ignored (1) in 2D */
    double vx, vy, vz;        /* voxel size [mm] */
    int32_t n_angles;         /* angles over [0, pi) */
    int32_t n_radial;         /* radial bins */
    double ds;                /* bin spacing [mm] */
    int32_t n_rings;          /* 3D: == nz */
    int32_t max_ring_diff;    /* 3D: D, span 1 */
    double ring_pitch;        /* 3D: == vz */
    double det_radius;        /* 3D: detector ring radius [mm], > image half-diagonal */
    int32_t n_subsets;        /* M, 1 <= M <= n_angles */
    /* The full 2D system model of Sec. IV-A (2D only; zeros = one line per
     * bin and no PSF).  A = diag(att) P B: P averages n_subrays parallel
     * sub-rays per bin, spread evenly over the bin width ds (offsets
     * ((k + 1/2)/n_subrays - 1/2) ds from the bin's line); B is a Gaussian
     * PSF of FWHM psf_fwhm applied in image space (taps at whole-pixel
     * distances up to ceil(3 sigma / v) <= 16 pixels, normalised per axis,
     * zero outside the image); att are per-bin attenuation factors given at
     * creation (pet_os_create_geometry_attenuated).  Geometries that use any
     * of them run through states and pet_os_reconstruct, not the batched or
     * served paths. */
    int32_t n_subrays;        /* 0 or 1: one line per bin; else 2..64 */
    double psf_fwhm;          /* [mm], 0: no PSF */
} pet_os_geom_desc;

/* Algorithm parameters (Sec. II, III-B, IV-A). */
typedef struct {
    int32_t mode;             /* PET_OS_BSREM .. PET_OS_P2, or PET_OS_OSEM */
    double beta;              /* >= 0, eq:ObjectiveFunction */
    double gamma_R;           /* >= 0, eq:RDP */
    double eps;               /* > 0, eq:RDP */
    double t_clip;            /* t of eq:OperatorPt, 0 < t < U */
    double U;                 /* box bound of eq:BoundedSet, > 0 */
    double lambda0, a;        /* lambda_k = lambda0/(a k + 1), both > 0 */
    double rho, delta1, delta2;  /* KM sequence, > 0 */
    double nu1, nu2;          /* clamp of nu, 0 < nu1 < nu2 */
    int64_t J0, J1;           /* 0 <= J0 <= J1, eq:nuki */
    int32_t objective_every;  /* reconstruct: objective each this many iterations (>= 1) */
} pet_os_params;

/* Human-readable message of the last failing call on this thread. */
const char* pet_os_last_error(void);

/* Library version string. */
const char* pet_os_version(void);

/* Geometry: validates the descriptor (Sec. IV-A conventions above), builds the
 * FP64 angle/bin/plane tables on the device and computes the sensitivity
 * s = A^T 1 and the normaliser p_j = s_j/M (or 1/M where s_j = 0) of eq:pj.
 * Size limits (PET_OS_ERR_INVALID_ARG beyond them): at most 2^30 voxels; one
 * pass of rays (3D: angle, bin, ring difference, 64-ring chunk items) below
 * 2^31; in 3D, max_ring_diff <= min(nz - 1, 31), nx nz and ny nz below 2^23,
 * and LORs no more oblique than one slice per transaxial voxel.
 * Synchronous.  The library owns *out until pet_os_destroy_geometry. */
int pet_os_create_geometry(const pet_os_geom_desc* desc, pet_os_geom** out);

/* The same with per-bin attenuation factors (Sec. IV-A: uniform water,
 * 0.096 / cm, over the object's support): att is a HOST array of n_bins
 * floats (natural layout, finite, > 0), copied; the model becomes
 * A = diag(att) P B, and the sensitivity A^T 1 includes it.  2D only. */
int pet_os_create_geometry_attenuated(const pet_os_geom_desc* desc, const float* att,
                                      pet_os_geom** out);

/* Attenuation factors att_i = exp(-sum_j a_ij mu_j) of the geometry's rays
 * through an attenuation map mu (DEVICE, n_voxels floats, per mm): the line
 * integrals of the sub-ray model P, without the PSF or any attenuation the
 * geometry already has.  att: DEVICE, n_bins floats.  Asynchronous. */
int pet_os_attenuation_factors(const pet_os_geom* geom, const float* mu, float* att,
                               pet_os_stream stream);
int pet_os_destroy_geometry(pet_os_geom* geom);

/* Sizes: voxels, bins (planes*angles*radial), planes. Any pointer may be NULL. */
int pet_os_geometry_info(const pet_os_geom* geom, int64_t* n_voxels, int64_t* n_bins,
                         int32_t* n_planes);

/* Copy of the sensitivity A^T 1 (eq:pj numerator) into out[n_voxels] (device). */
int pet_os_sensitivity(const pet_os_geom* geom, float* out, pet_os_stream stream);

/* q = A_i f: forward projection (sec. II-B) of the rays of subset `subset`
 * (1..M), or of every ray when subset == 0.  q is natural layout; entries of
 * other subsets are not written.  f: n_voxels floats, q: n_bins floats. */
int pet_os_forward(const pet_os_geom* geom, const float* f, int32_t subset, float* q,
                   pet_os_stream stream);

/* out = A_i^T w: back-projection of the rays of `subset` (0 = all), w in
 * natural layout (entries of other subsets ignored).  Voxel-driven gather,
 * no atomics, deterministic. */
int pet_os_back(const pet_os_geom* geom, const float* w, int32_t subset, float* out,
                pet_os_stream stream);

/* Objective Phi(f) of eq:ObjectiveFunction (fidelity eq:FidelityTerm with
 * FP64 log and sums, plus beta R(f)).  Synchronous: *phi is a host double. */
int pet_os_objective(const pet_os_geom* geom, const pet_os_params* params, const float* f,
                     const float* y, const float* r, double* phi, pet_os_stream stream);

/* Default box bound (the paper only proves U exists, eq:BoundedSet):
 * U = 1e3 * max(max_j f0_j, (sum y - sum r)_+ / sum_j s_j).  Synchronous. */
int pet_os_default_U(const pet_os_geom* geom, const float* f0, const float* y, const float* r,
                     double* U, pet_os_stream stream);

/* Subset gradient of Sec. II-B: grad Phi_i(f) = A_i^T (1 - y_i/(A_i f + r_i))
 * + (beta/M) grad R(f) for subset i in 1..M, or grad Phi(f) (every ray, full
 * weight beta) when subset == 0.  Only params->beta, gamma_R and eps are
 * used.  f, grad: n_voxels floats (device, natural layout); y, r: n_bins
 * floats.  Scratch is allocated and released inside; synchronous. */
int pet_os_subset_gradient(const pet_os_geom* geom, const pet_os_params* params, const float* f,
                           const float* y, const float* r, int32_t subset, float* grad,
                           pet_os_stream stream);

/* Gradient-consistency measure of Sec. IV-B (Fig. 2): with m = mean(f) and
 * grad(f) the gradient magnitude of the smoothness measure (Sec. III-B), the
 * smooth area I_s = {j : grad(f)_j < smooth_frac m} and the variable area
 * I_v = {j : grad(f)_j > var_frac m} (the paper uses 0.01 and 0.2; both
 * decisions in FP64), and the angle arccos(<u, v>/(|u| |v|)) between
 * h_prev and h_cur restricted to each area, in radians (NaN when the area
 * is empty or either restriction is zero).  theta: HOST double[2] (smooth,
 * variable); count: HOST int64[2] (|I_s|, |I_v|) or NULL.  h_prev, h_cur,
 * f: n_voxels floats (device).  Sums in FP64 in a fixed order (bitwise
 * reproducible).  Scratch is allocated and released inside; synchronous. */
int pet_os_gradient_angles(const pet_os_geom* geom, const float* h_prev, const float* h_cur,
                           const float* f, double smooth_frac, double var_frac, double* theta,
                           int64_t* count, pet_os_stream stream);

/* Per-reconstruction state: position (k, i) of the next subiteration, the
 * Nesterov t (FP64), the frozen nu of eq:nuki, and device scratch.  `params`
 * is copied and validated.  The geometry must outlive the state. */
int pet_os_state_create(const pet_os_geom* geom, const pet_os_params* params,
                        pet_os_state** out);
int pet_os_state_destroy(pet_os_state* state);

/* Position of the next subiteration: k (0-based iteration), i (1-based subset). */
int pet_os_state_position(const pet_os_state* state, int64_t* k, int32_t* i);

/* One subiteration of Table I on f (in place, n_voxels floats, device):
 *   q = A_i f; w = 1 - y_i/(q + r_i); b = A_i^T w;  grad Phi_i = b + (beta/M) grad R(f)
 *   f~ = f - lambda_k alpha_{k,i} nu^{k,i} S(f) grad Phi_i;  f = P_t(f~)
 * then advances (k, i).  nu^{k,i} is computed from the iterate entering the
 * subiteration.  y, r: n_bins floats (natural layout, r > 0).  Asynchronous;
 * the FP64 scalars lambda_k, alpha_{k,i} are evaluated on the host.  The
 * first call with a (f, y, r) triple makes the data check (conventions). */
int pet_os_subiteration(pet_os_state* state, float* f, const float* y, const float* r,
                        pet_os_stream stream);

/* n_iter iterations (n_iter * M subiterations) of SDP-BSREM from f (in/out).
 * obj: NULL, or a HOST array of n_iter+1 doubles receiving Phi(f^k) for
 * k = 0, objective_every, 2*objective_every, ... (other entries NaN); the
 * call then blocks at the end.  The data check (conventions) runs first and
 * waits for `stream`; with obj == NULL the iterations are queued
 * asynchronously after it. */
int pet_os_reconstruct(const pet_os_geom* geom, const pet_os_params* params, float* f,
                       const float* y, const float* r, int32_t n_iter, double* obj,
                       pet_os_stream stream);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): pet_os_reconstruct with obj == NULL, the
 * same kernels and the same result bit for bit, with the request's scratch
 * (subset sinogram, gradient, mu, nu, iterate copy, FP64 partials) placed in
 * a static device array of PET_OS_NOALLOC_SCRATCH_BYTES that every GPU the
 * library runs on holds until the process ends, instead of allocated memory.
 * It calls no device allocation routine.  Arguments as pet_os_reconstruct;
 * the geometry must belong to the current device.  Errors: INVALID_ARG also
 * when the request's scratch exceeds the array (the message states both
 * sizes; a 200x200x64 volume with 224 x 281 x 1744 bins and 28 subsets needs
 * about 75 MB) and for PET_OS_OSEM (its subset sensitivities need a state).
 * The data check (conventions) waits for `stream` before the iterations are
 * queued; the iterations run asynchronously.  Every call on a GPU shares that
 * GPU's array and overwrites what the previous call left there: calls queued
 * on one stream run one after the other, calls that overlap on one GPU
 * (different streams or threads) race and must not be made. */
#define PET_OS_NOALLOC_SCRATCH_BYTES (96u << 20)
int pet_os_reconstruct_noalloc(const pet_os_geom* geom, const pet_os_params* params, float* f,
                               const float* y, const float* r, int32_t n_iter, pet_os_stream stream);

/* n_iter further iterations (n_iter * M subiterations) on an existing state,
 * from its current position, on f (in/out).  Uses only the state's scratch
 * (no allocation).  obj: NULL, or a HOST array of n_iter doubles receiving
 * Phi after iteration j+1 when (j+1) % objective_every == 0 or j+1 == n_iter
 * (NaN otherwise); the call then blocks at the end.  Asynchronous otherwise. */
int pet_os_run(pet_os_state* state, float* f, const float* y, const float* r, int32_t n_iter,
               double* obj, pet_os_stream stream);

/* Kernel timing with HIP events on the state's stream (tracing, Sec. IV
 * reports CPU time; this reports device time).  kernel: 0 = forward
 * projection + ratio, 1 = back-projection (2D: with the RDP/mu stencil and
 * the update; 3D: with the RDP gradient and mu blocks in the same launch),
 * 2 = 3D update, 3 = accepted and brackets nothing (the 3D RDP gradient has
 * no launch of its own in a subiteration), -1 = off.  Events bracket every
 * launch of that kernel until switched off.
 * read: synchronises, returns the summed milliseconds and launch count since
 * the last read, and resets them. */
int pet_os_state_profile(pet_os_state* state, int32_t kernel);
int pet_os_state_profile_read(pet_os_state* state, double* total_ms, int64_t* launches);

/* Number of nonzero a_ij of subset `subset` (0 = all rays): the work of one
 * projection in the system model.  Synchronous. */
int pet_os_nnz(const pet_os_geom* geom, int32_t subset, int64_t* nnz);

/* Position a state at subiteration (k, i) with Nesterov t = t_nest (>= 1) and,
 * when nu_frozen (DEVICE, n_voxels floats) is not NULL, the frozen nu of
 * eq:nuki (P1/P2 only; marks it present).  Used to resume from state held
 * elsewhere.  Synchronous with respect to the device copy. */
int pet_os_state_seek(pet_os_state* state, int64_t k, int32_t i, double t_nest, const float* nu_frozen);

/* Checkpoint of a state: (k, i, t, params, geometry descriptor, frozen nu).
 * export: buf == NULL queries the size into *len; otherwise *len must be at
 * least that size.  Synchronous (copies the frozen nu to the host).
 * import: the target state must have the same geometry descriptor and mode,
 * else PET_OS_ERR_STATE_MISMATCH; the checkpoint's parameters, position and
 * Nesterov t must pass the checks of pet_os_state_create and
 * pet_os_state_seek, and a frozen nu is accepted only by a P1/P2 state
 * (INVALID_ARG, with the state unchanged).  The next subiteration makes the
 * data check again (U may have changed). */
int pet_os_state_export(const pet_os_state* state, void* buf, size_t* len);
int pet_os_state_import(pet_os_state* state, const void* buf, size_t len);

/* ------------------------------------------------------------------------
 * Batched execution: many independent reconstructions of different sizes
 * advanced together.  Every step advances each active request by one
 * subiteration (Table I) with one persistent launch per kernel, over a
 * device-resident work list of (request, block) items; the launch sequence
 * is captured once in a hipGraph and replayed.  A request computes exactly
 * what pet_os_reconstruct computes for it alone (same kernels, same
 * reductions); the FP64 scalar schedule of every subiteration is evaluated on
 * the host when the request is added.
 * ------------------------------------------------------------------------ */
typedef struct pet_os_batch pet_os_batch;

/* A batch with room for max_slots concurrent requests (1..65536). */
int pet_os_batch_create(int32_t max_slots, pet_os_batch** out);
/* Waits for the device, frees every slot and the batch. */
int pet_os_batch_destroy(pet_os_batch* batch);

/* Admit a request: n_iter iterations of SDP-BSREM from f (in/out, device)
 * with data y, r (device, natural layout) on `geom` (must outlive the slot).
 * Allocates the request's scratch and schedule, queues sum(f) on `stream`;
 * synchronises `stream` first (the slot table is read by queued steps).
 * Errors: INVALID_ARG (also data that fail the check of the conventions),
 * BUDGET (no free slot), OUT_OF_MEMORY. */
int pet_os_batch_add(pet_os_batch* batch, const pet_os_geom* geom, const pet_os_params* params, float* f,
                     const float* y, const float* r, int32_t n_iter, pet_os_stream stream, int32_t* slot);
/* Release a slot (synchronises `stream`); its f holds the last iterate. */
int pet_os_batch_remove(pet_os_batch* batch, int32_t slot, pet_os_stream stream);
/* Queue n_steps batched subiterations on `stream` (asynchronous).  After
 * slots joined or left, the first step rebuilds the work lists and captures
 * a new graph (on a private stream, thread-local capture mode).  A capture
 * fails if another thread issues default-stream (NULL-stream) work at the
 * same time, so a program that drives batches and other pet_os calls from
 * several threads serializes those calls (the server does). */
int pet_os_batch_step(pet_os_batch* batch, int32_t n_steps, pet_os_stream stream);
/* Queue as many steps as the longest active request still needs. */
int pet_os_batch_run(pet_os_batch* batch, pet_os_stream stream);
/* Host view of a slot: active (1 while subiterations remain) and the number
 * of subiterations still to run once the queued steps complete. */
int pet_os_batch_slot_status(const pet_os_batch* batch, int32_t slot, int32_t* active, int64_t* remaining);
/* Device bytes held by the batch's slots (scratch and schedules). */
int pet_os_batch_bytes(const pet_os_batch* batch, size_t* bytes);

/* n requests (arrays of n geometries, parameter sets, f, y, r pointers and
 * iteration counts) reconstructed in one batch; blocks until done. */
int pet_os_reconstruct_batch(int32_t n, const pet_os_geom* const* geoms, const pet_os_params* params,
                             float* const* f, const float* const* y, const float* const* r,
                             const int32_t* n_iter, pet_os_stream stream);

/* Autotuner: times the forward projector's threads per ray (1, 4, 16, 64) and,
 * in 2D, the back-projector's tile (16x16, or 8x8 with four angle groups) on
 * this geometry's first subset and keeps the fastest for all later launches
 * with this geometry (plain and batched).  In 3D it times the single-request
 * back-projector's slices per block (16, 32, 64) and ring differences staged
 * together (4, 8) instead; batched 3D launches keep their fixed shape.  The
 * default shape is timed first and another replaces it only when at least
 * 3 % faster.  flags bit 0: ignore the cache.
 * When the environment variable PET_OS_TUNE_CACHE names a file, results are
 * read from / appended to it keyed by the geometry descriptor.  Synchronous. */
int pet_os_autotune(pet_os_geom* geom, int32_t flags, pet_os_stream stream);
/* The projector shapes the single-request launches of this geometry use now
 * (current[4], after any autotuning) and the defaults they start from
 * (defaults[4]), each as {forward-projector threads per ray (2D; 0 in 3D),
 * back-projector tile kind (2D: 0 = 16x16, 1 = 8x8 with four angle groups;
 * 3D: 2), 3D slices per block, 3D ring differences per staging group (0 in
 * 2D)}.  Host only; either array may be NULL. */
int pet_os_geometry_shapes(const pet_os_geom* geom, int32_t* current, int32_t* defaults);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of reconstruction requests.  2D and 3D
 * requests have a lane each (batch, stream, worker thread), running
 * concurrently on the device.  A lane admits the queued requests of its class
 * in arrival order whenever a slot is free (max_slots counts both lanes) and
 * the device memory they need (scratch, schedule, and their geometry if not
 * cached) fits the shared budget; admitted requests join the lane's running
 * batch between two batched subiterations and leave it as soon as they
 * finish.  Geometries (tables, sensitivity, autotuned shapes) are cached by
 * descriptor and counted against the budget; unused ones are evicted first.
 * The caller's f, y, r buffers are not counted.
 * ------------------------------------------------------------------------ */
typedef struct pet_os_server pet_os_server;

typedef struct {
    pet_os_geom_desc desc;     /* geometry of the request */
    pet_os_params params;      /* algorithm parameters (validated at submit) */
    float* f;                  /* DEVICE: f0 in, result out; valid until the ticket completes */
    const float* y;            /* DEVICE counts, natural layout */
    const float* r;            /* DEVICE background, natural layout */
    int32_t n_iter;            /* iterations (>= 1) */
    int32_t want_objective;    /* nonzero: Phi(f) after the last iteration in the result */
} pet_os_request;

typedef struct {
    int32_t status;            /* PET_OS_OK or an error code (BUDGET, NUMERIC, DEVICE, TIMEOUT = cancelled) */
    int32_t pad;
    double objective;          /* Phi of the result, NaN if not requested */
    double t_submit, t_admit, t_start, t_finish;   /* seconds since the server was created */
    int64_t subiterations;     /* subiterations run */
    char message[128];         /* reason when status != PET_OS_OK */
} pet_os_result;

typedef struct {
    int64_t queued, active, ticks, max_active;
    size_t bytes_in_use;
    int64_t geometries_cached;
} pet_os_server_stats_t;

/* A server on the current device with its own streams; hbm_budget_bytes caps
 * the device memory it allocates, max_slots the concurrent requests. */
int pet_os_server_create(size_t hbm_budget_bytes, int32_t max_slots, pet_os_server** out);
/* Finishes every queued and running request, then stops. */
int pet_os_server_destroy(pet_os_server* server);
/* Queue a request; returns at once with a ticket.  Invalid descriptors,
 * parameters or pointers are rejected synchronously (INVALID_ARG).  The data
 * (y, r, f0) are checked at admission (conventions); a request whose data
 * fail ends with status INVALID_ARG and the others are not affected. */
int pet_os_submit(pet_os_server* server, const pet_os_request* req, uint64_t* ticket);
/* Wait up to timeout_us (< 0: forever) for a ticket; fills *out and releases
 * the ticket.  PET_OS_ERR_TIMEOUT if it is still running. */
int pet_os_wait(pet_os_server* server, uint64_t ticket, int64_t timeout_us, pet_os_result* out);
/* Ask for a request to be dropped (before admission, or at the next step). */
int pet_os_cancel(pet_os_server* server, uint64_t ticket);
int pet_os_server_stats(pet_os_server* server, pet_os_server_stats_t* out);

/* Host-only server for tests of scheduling and failure handling: no device
 * calls are made (data pointers may be NULL); a batched step takes step_us of
 * wall time.  pet_os_server_inject arms faults on the lane of 2D requests. */
int pet_os_server_create_simulated(size_t budget_bytes, int32_t max_slots, int64_t step_us, pet_os_server** out);
#define PET_OS_INJECT_ADMIT_OOM 1      /* the next admissions fail with OUT_OF_MEMORY */
#define PET_OS_INJECT_STEP_FAILURE 2   /* the next batched steps fail (DEVICE) */
#define PET_OS_INJECT_NAN_OBJECTIVE 3  /* the next objectives come back NaN */
#define PET_OS_INJECT_BAD_DATA 4       /* the next admissions fail the data check (INVALID_ARG) */
int pet_os_server_inject(pet_os_server* server, int32_t kind, int32_t count);

#ifdef __cplusplus
}
#endif
#endif /* PET_OS_H */
