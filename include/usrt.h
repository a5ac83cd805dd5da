/*
 * usrt.h — C-ABI of the MI355X (gfx950) library for differentiable full-path
 * Monte-Carlo ultrasound ray tracing ("Fully Differentiable Ultrasound
 * Simulation Utilizing Ray-Tracing", arXiv 2604.15017).
 *
 * Conventions shared by every entry point
 *  - Return value: 0 (US_OK) on success, a negative US_E* code otherwise; the
 *    message of the last failure on the calling thread is us_last_error().
 *    Argument errors are detected on the host before anything is launched.
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t passed as a
 *    plain pointer; NULL = the device's null stream). Device faults surface on
 *    a later call or on stream synchronisation.
 *  - Pointers named *_dev are device memory owned by the caller; the library
 *    never frees them. Descriptors and host arrays are read during the call
 *    only. Handles (us_ctx, us_probe, us_scene) are owned by the library until
 *    their destroy call; they hold resident device copies of what was uploaded.
 *  - Scratch: every compute entry point takes a caller-allocated device
 *    workspace `ws_dev` of `ws_bytes`, whose required size the matching
 *    *_workspace_size() call returns; the library allocates nothing during
 *    compute calls. Calls sharing a workspace must be ordered on one stream.
 *  - Units: metres, seconds, hertz, m/s, MRayl, dB/cm/MHz, radians.
 *  - Layouts (row-major, last index fastest):
 *      rf        float  [n_tx][n_elem][n_t]
 *      iq        float  [n_x][n_z][2]  (real, imaginary)
 *      bmode     float  [n_x][n_z]     (dB, in [-dr_db, 0])
 *      theta     double [n_params]: (c, Z, alpha) per region, then plane
 *                depths, then (cx, cy, cz, r) per sphere, then (cx, cz, R)
 *                per cylinder, then the GGX roughness of every plane,
 *                sphere, cylinder and mesh (>= 0; 0 is a mirror), then the
 *                displacement coefficients q[mesh][j] of the meshes
 */
#ifndef USRT_H
#define USRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  US_OK = 0,
  US_EINVAL = -1,   /* bad argument (sizes, layout, pointers) */
  US_ENOMEM = -2,   /* device allocation failed (handle creation only) */
  US_EDEVICE = -3,  /* a HIP runtime call failed */
  US_ETOOBIG = -4,  /* workspace smaller than required */
};

typedef struct us_ctx us_ctx;
typedef struct us_probe us_probe;
typedef struct us_scene us_scene;

/* Linear array on z = 0 facing +z (Sec. 2.3.1): element e centred at
 * x_e = (e - (n_elem - 1)/2) pitch; receive directivity of Eq. cutoff with
 * main-lobe angle alpha_main and cutoff alpha_cut; pulse of Eq. axial_sig at
 * f0 with an envelope n_cycles / f0 wide at half maximum; n_t samples at fs;
 * c_ref is the sound speed of the steering and beamforming delays. */
typedef struct us_probe_desc {
  int32_t n_elem;
  double pitch, elem_width, elem_height;
  double f0, n_cycles, fs;
  int32_t n_t;
  double c_ref, alpha_main, alpha_cut;
} us_probe_desc;

/* Scene of homogeneous regions bounded by planes z = d, spheres, cylinders
 * along the elevation axis y ((x - cx)^2 + (z - cz)^2 = R^2, the hollow
 * cylinder of the paper's forward check and inversions) and closed triangle
 * meshes (Sec. 2.3.2; meshes as in the anatomy scenes of Sec. 4).
 * theta holds the continuous parameters (layout above); plane_regions[k] =
 * {region above, region below}; sphere_regions[k] and mesh_regions[m] =
 * {inside, outside}; kd = fraction of the reflected energy scattered into the
 * Lambertian lobe; start_region = region at the array face. Host arrays.
 * Roughness rho (Eq. GGX_PDF): the specular share (1 - kd) of the reflection
 * is mirrored about a microfacet normal drawn from the GGX distribution with
 * density D(m) (n.m), weighted by the Smith-masked microfacet estimator
 * G1(i) G1(o) |i.m| / ((n.i) (n.m)); a glossy path reaches the elements
 * directly (no secondary ray), a reflection below the surface ends it.
 *
 * Meshes (n_meshes = 0: none, and the mesh pointers may be NULL): the
 * vertices of all meshes are concatenated in mesh order ([n_vertices][3]
 * rest positions, owning mesh vmesh[v], non-decreasing), and so are the
 * triangles ([n_triangles][3] global
 * vertex ids, counter-clockwise seen from outside, owning mesh tmesh[t], all
 * three vertices of that mesh). Vertex v moves along its unit direction
 * vnormal[v] by sum_j q[vmesh[v]][j] vbasis[v][j]; faces are flat. At most
 * 32 meshes and 2^27 - 1 triangles; zero-area triangles are rejected. The library builds a
 * 4-wide bounding-volume hierarchy on upload (rejected with US_EINVAL if too
 * deep: its binary form over 38 levels, or over 20 levels of 4-wide nodes)
 * and refits it on every us_scene_set_params. */
typedef struct us_scene_desc {
  int32_t n_regions, n_planes, n_spheres;
  const double* theta;
  const int32_t* plane_regions;
  const double* plane_kd;
  const int32_t* sphere_regions;
  const double* sphere_kd;
  int32_t start_region;
  int32_t n_meshes, n_basis;
  const int32_t* mesh_regions;   /* [n_meshes][2] */
  const double* mesh_kd;         /* [n_meshes] */
  int64_t n_vertices, n_triangles;
  const double* vertices;        /* [n_vertices][3] */
  const double* vnormal;         /* [n_vertices][3] */
  const double* vbasis;          /* [n_vertices][n_basis] */
  const int32_t* vmesh;          /* [n_vertices] */
  const int32_t* triangles;      /* [n_triangles][3] */
  const int32_t* tmesh;          /* [n_triangles] */
  int32_t n_cylinders;           /* at most 16; axis along y through (x, z) of theta */
  const int32_t* cylinder_regions;   /* [n_cylinders][2]: inside, outside */
  const double* cylinder_kd;         /* [n_cylinders] */
} us_scene_desc;

/* One plane-wave transmit: steering angle and the id that seeds its rays. */
typedef struct us_tx_desc {
  double angle;
  uint32_t id;
} us_tx_desc;

/* Pixel centres x_a = x0 + a dx, z_b = z0 + b dz (z > 0 below the array). */
typedef struct us_grid_desc {
  int32_t n_x, n_z;
  double x0, dx, z0, dz;
} us_grid_desc;

/* Last error message of the calling thread ("" if none). */
const char* us_last_error(void);

/* Context bound to one HIP device. Probes and scenes keep their device and
 * may be destroyed before or after their context (compute calls need it
 * alive). Every call that launches work makes the context's device current
 * and first clears the HIP runtime's last-error state of the calling thread,
 * so that it reports only its own launch failures. */
int us_create(int device, us_ctx** out);
int us_destroy(us_ctx* ctx);

/* Uploads a probe (resident pulse taps and FFT twiddles). */
int us_probe_upload(us_ctx* ctx, const us_probe_desc* desc, us_probe** out);
int us_probe_destroy(us_probe* probe);

/* Uploads a scene; *n_params receives the length of theta. */
int us_scene_upload(us_ctx* ctx, const us_scene_desc* desc, us_scene** out, int32_t* n_params);
int us_scene_destroy(us_scene* scene);
/* Replaces the scene's resident theta with n_params doubles from device
 * memory theta_dev (asynchronous copy on stream); with meshes, also moves
 * the vertices and refits the hierarchy on stream. */
int us_scene_set_params(us_scene* scene, const double* theta_dev, int32_t n_params, void* stream);

/* Forward transport, Sec. 2.3 (emission, traversal with Snell reflection /
 * refraction / Lambertian backscatter / GGX glossy reflection, attenuation, receiver-directed
 * secondary rays, time-of-flight deposit with a linear tent, Eq. axial_sig
 * pulse filter). Traces rays [ray_begin, ray_begin + ray_count) of each of
 * the n_tx transmits (ray id = element * rays_per_elem + j, Philox4x64-10
 * counter (ray id, tx.id, event, 0), key (seed, 0)); each ray has weight
 * 1/rays_per_elem so disjoint ray ranges add up.
 *   rf_dev        out: float [n_tx][n_elem][n_t] (overwritten)
 *   counters_dev  optional (NULL): int64 [5], accumulated: primary segments,
 *                 secondary-ray segments, deposits, interactions, secondary
 *                 rays traced (a segment is one closest-hit query)
 *   ray_hash_dev  optional (NULL): uint64 [n_tx][ray_count], overwritten with
 *                 each ray's decision hash (sum over its events of SplitMix64
 *                 of (tag, event, word)), for auditing branch agreement
 *   max_bounces   at most this many interactions per path (>= 0) */
size_t us_simulate_rf_workspace_size(const us_scene* scene, const us_probe* probe, int32_t n_tx,
                                     int64_t ray_count, int32_t max_bounces);
int us_simulate_rf(us_ctx* ctx, const us_scene* scene, const us_probe* probe,
                   const us_tx_desc* tx, int32_t n_tx, uint64_t seed, int32_t rays_per_elem,
                   int64_t ray_begin, int64_t ray_count, int32_t max_bounces, float* rf_dev,
                   int64_t* counters_dev, uint64_t* ray_hash_dev, void* ws_dev, size_t ws_bytes,
                   void* stream);

/* Plane-wave delay-and-sum, Eq. das: analytic signal of each RF channel along
 * time (demodulation, Sec. 2.3.4), then I(x, z) = sum over transmits and
 * elements of the linearly interpolated analytic sample at
 * fs (x sin th + z cos th + |(x, z) - (x_e, 0)|) / c_ref, unit weights,
 * samples outside [0, n_t) read as zero. n_t must be a power of two in
 * [64, 8192].
 *   rf_dev in: float [n_tx][n_elem][n_t]; iq_dev out: float [n_x][n_z][2] */
size_t us_beamform_workspace_size(const us_probe* probe, int32_t n_tx);
int us_beamform(us_ctx* ctx, const us_probe* probe, const us_grid_desc* grid,
                const us_tx_desc* tx, int32_t n_tx, const float* rf_dev, float* iq_dev,
                void* ws_dev, size_t ws_bytes, void* stream);

/* us_beamform for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same result, with the analytic signal kept in a
 * file-scope device array of the library instead of a workspace. The array
 * holds at most 64 MiB (8,388,608 complex samples: n_tx * n_elem * n_t of
 * them; US_ETOOBIG beyond, with nothing launched); each GPU that loads the
 * library holds its own copy until the process ends. Allocates nothing and
 * clears nothing (every sample it reads is written first in the same call).
 * All calls on one GPU share its array: calls that overlap in time on one
 * GPU (on different streams, or from different threads) race and give wrong
 * results; serialise them. */
int us_beamform_static(us_ctx* ctx, const us_probe* probe, const us_grid_desc* grid,
                       const us_tx_desc* tx, int32_t n_tx, const float* rf_dev, float* iq_dev,
                       void* stream);

/* Envelope and log compression (Sec. 2.3.4, Sec. 3.1):
 * bmode = max(20 log10(|iq| / max|iq|), -dr_db). */
size_t us_bmode_workspace_size(int64_t n_px);
int us_bmode(us_ctx* ctx, const float* iq_dev, int64_t n_px, float dr_db, float* bmode_dev,
             void* ws_dev, size_t ws_bytes, void* stream);

/* Image-space loss (Sec. 3.5, Eq. weighted_l1_l2_loss):
 * L = (1/n_px) sum_u [lambda1 |B_u - R_u| + lambda2 (B_u - R_u)^2]; the mean
 * squared error is lambda1 = 0, lambda2 = 1.
 *   loss_dev out: double [1] (overwritten); summed in integer windows, so
 *     the value does not depend on the order in which blocks finish
 *   g_bmode_dev optional out (NULL): float [n_px], dL/dB (sign(0) = 0)
 *   ws_dev: device workspace of us_image_loss_workspace_size(n_px) bytes
 *     (US_ETOOBIG if smaller, US_EINVAL if NULL) */
size_t us_image_loss_workspace_size(int64_t n_px);
int us_image_loss(us_ctx* ctx, const float* bmode_dev, const float* ref_dev, int64_t n_px,
                  double lambda1, double lambda2, double* loss_dev, float* g_bmode_dev,
                  void* ws_dev, size_t ws_bytes, void* stream);

/* Vector-Jacobian products (Sec. 3.2-3.3). */
/* g_iq = (d bmode / d iq)^T g_bmode, including the normalisation by the
 * frame maximum (first largest pixel); clipped pixels contribute nothing.
 *   g_iq_dev out: float [n_x][n_z][2] (d/dRe, d/dIm) */
int us_bmode_vjp(us_ctx* ctx, const float* iq_dev, const float* g_bmode_dev, int64_t n_px,
                 float dr_db, float* g_iq_dev, void* ws_dev, size_t ws_bytes, void* stream);
/* g_rf = adjoint of us_beamform (Eq. das_adjoint, then the self-adjoint
 * analytic-signal map, real part). Computed per RF row in LDS, the image
 * walked column by column (a column's pixels touch disjoint sample pairs
 * when the grid's rows are more than two samples apart), else per RF sample
 * as a gather over the pixels that interpolate from it; no atomics either
 * way, so the result does not depend on scheduling.
 *   g_iq_dev in: float [n_x][n_z][2]; g_rf_dev out: float [n_tx][n_elem][n_t] */
size_t us_beamform_vjp_workspace_size(const us_probe* probe, int32_t n_tx);
int us_beamform_vjp(us_ctx* ctx, const us_probe* probe, const us_grid_desc* grid,
                    const us_tx_desc* tx, int32_t n_tx, const float* g_iq_dev, float* g_rf_dev,
                    void* ws_dev, size_t ws_bytes, void* stream);
/* Gradients of Re<g_iq, I>, I the image us_beamform forms from rf_dev, with
 * respect to the acquisition parameters of Eq. das at fixed RF: the steering
 * angle of each transmit (radians), the speed of sound c_ref of the delays
 * (m/s) and the element pitch (m). I depends on them only through the
 * fractional sample index fs tau, and the linear interpolation's slope in it
 * is A[k0 + 1] - A[k0] (A the analytic signal). Sums in fp64 in a fixed
 * order (the result does not depend on scheduling).
 *   rf_dev in: float [n_tx][n_elem][n_t]; g_iq_dev in: float [n_x][n_z][2]
 *   g_acq_dev out: double [n_tx + 2] (overwritten): d/d angle of each
 *   transmit, then d/d c_ref, then d/d pitch
 * The workspace depends on the grid (partial sums per tile of 256 pixels). */
size_t us_beamform_acq_vjp_workspace_size(const us_probe* probe, const us_grid_desc* grid, int32_t n_tx);
int us_beamform_acq_vjp(us_ctx* ctx, const us_probe* probe, const us_grid_desc* grid,
                        const us_tx_desc* tx, int32_t n_tx, const float* rf_dev, const float* g_iq_dev,
                        double* g_acq_dev, void* ws_dev, size_t ws_bytes, void* stream);
/* g_theta += (d rf / d theta)^T g_rf at fixed ray realizations (Sec. 3.2,
 * Eq. chain_rule): the paths of the same rays as us_simulate_rf are replayed
 * from their Philox counters (nothing stored between the calls); discrete
 * choices are frozen and branch probabilities are not differentiated.
 *   g_rf_dev in: float [n_tx][n_elem][n_t]; g_theta_dev in/out: double [n_params]
 *   ws_dev: the workspace size for the call's ray_count lets the replay take
 *   all rays in chunks of up to 2^23; a smaller one, down to the size for
 *   ray_count = 1 (US_ETOOBIG below it), shortens the chunks to what fits.
 *   The result does not depend on it. */
size_t us_simulate_rf_vjp_workspace_size(const us_scene* scene, const us_probe* probe,
                                         int32_t n_tx, int64_t ray_count, int32_t max_bounces);
int us_simulate_rf_vjp(us_ctx* ctx, const us_scene* scene, const us_probe* probe,
                       const us_tx_desc* tx, int32_t n_tx, uint64_t seed, int32_t rays_per_elem,
                       int64_t ray_begin, int64_t ray_count, int32_t max_bounces,
                       const float* g_rf_dev, double* g_theta_dev, void* ws_dev, size_t ws_bytes,
                       void* stream);
/* us_simulate_rf_vjp, and also the gradient of the same contraction with
 * respect to the acquisition parameters, at the same fixed ray realizations:
 * the steering angle of each transmit (emission direction, emission delay
 * x sin th / c_ref, weight cos th / rays_per_elem), c_ref (emission delay)
 * the pitch (element centres of the emission origins and of the
 * receiver-directed rays' targets) and the centre frequency f0 (the pulse of
 * Eq. axial_sig, carrier and envelope width n_cycles / f0, and the amplitude
 * attenuation alpha f0 of every region; the tap count M is held fixed). Which
 * element an array hit lands on is piecewise constant in the pitch and not
 * differentiated. The workspace is that of us_simulate_rf_vjp.
 *   g_acq_dev in/out: double [n_tx + 3], accumulated: d/d angle of each
 *   transmit, then d/d c_ref, d/d pitch and d/d f0 (summed in integer
 *   windows, so the values do not depend on scheduling) */
int us_simulate_rf_vjp_acq(us_ctx* ctx, const us_scene* scene, const us_probe* probe,
                           const us_tx_desc* tx, int32_t n_tx, uint64_t seed, int32_t rays_per_elem,
                           int64_t ray_begin, int64_t ray_count, int32_t max_bounces,
                           const float* g_rf_dev, double* g_theta_dev, double* g_acq_dev, void* ws_dev,
                           size_t ws_bytes, void* stream);

/* The backward of one frame in one call, from dL/dB to g_theta (Sec. 3.2-3.3,
 * Eq. das_adjoint, Eq. chain_rule): us_bmode_vjp, then us_beamform_vjp, then
 * us_simulate_rf_vjp, with the image and analytic-signal gradients kept in
 * the workspace and the analytic-signal adjoint and the pulse adjoint run as
 * one kernel per RF row (dL/drf stays in LDS and never reaches HBM). The
 * arithmetic is that of the three calls in the same order: g_theta is bit for
 * bit the three-call result.
 *   iq_dev in: float [n_x][n_z][2], the image the B-mode frame came from
 *   (us_beamform of the same scene, probe, transmits and grid)
 *   g_bmode_dev in: float [n_x][n_z], dL/dB; dr_db as for us_bmode
 *   g_theta_dev in/out: double [n_params], accumulated
 *   ws_dev: us_frame_vjp_workspace_size(...) bytes for the call's ray_count
 *   let the replay take all rays in chunks of up to 2^23; a smaller
 *   workspace, down to the size for ray_count = 1 (US_ETOOBIG below it),
 *   shortens the chunks to what fits. The result does not depend on it.
 * Arguments are checked as for the three calls (US_EINVAL). */
size_t us_frame_vjp_workspace_size(const us_scene* scene, const us_probe* probe, const us_grid_desc* grid,
                                   int32_t n_tx, int64_t ray_count, int32_t max_bounces);
int us_frame_vjp(us_ctx* ctx, const us_scene* scene, const us_probe* probe, const us_grid_desc* grid,
                 const us_tx_desc* tx, int32_t n_tx, uint64_t seed, int32_t rays_per_elem, int64_t ray_begin,
                 int64_t ray_count, int32_t max_bounces, const float* iq_dev, const float* g_bmode_dev,
                 float dr_db, double* g_theta_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* Recorded frame: a forward that keeps the replay's step records for the
 * backward that follows it (Sec. 3.2 differentiates the path of fixed random
 * numbers; the backward of a recorded frame reads the path instead of tracing
 * it again), trading device memory (about 3 KB per ray at twelve
 * interactions: step records, the replay's scratch and each receiver
 * segment's march) for the replay's forward phase and its marches.
 *
 * us_simulate_rf_recorded computes the RF of us_simulate_rf for the same
 * arguments, bit for bit (the same fp64 path arithmetic, the same integer
 * histogram; counters_dev, optional (NULL), accumulates the same event
 * counts), and leaves in ws_dev the step record of every segment, the
 * diffuse interactions in the receiver segments' key order and the per-step
 * counts. One launch group only (n_tx <= 64) and ray_count >= 1, all
 * n_tx * ray_count rays in one chunk: ws_dev must hold
 * us_recorded_workspace_size(...) bytes (US_ETOOBIG if smaller; 0 from the
 * size function for n_tx > 64 or ray_count < 1). The scene remembers the
 * call (workspace and arguments, host side only); us_scene_set_params on the
 * scene invalidates the records.
 *
 * us_simulate_rf_vjp_recorded and us_frame_vjp_recorded then give exactly the
 * gradient of us_simulate_rf_vjp and us_frame_vjp (bit for bit) from those
 * records: they must be called with the same scene (parameters unchanged),
 * probe, transmits, seed, rays per element, ray range and bounces, and the
 * same workspace untouched since (rec_dev, rec_bytes for the frame call),
 * else US_EINVAL before anything is launched. The records stay valid, so
 * several backward calls may follow one forward. us_frame_vjp_recorded takes
 * a second workspace ws_dev for the image adjoint's buffers,
 * us_frame_vjp_recorded_workspace_size(...) bytes. Calls that share a
 * workspace must not overlap. */
size_t us_recorded_workspace_size(const us_scene* scene, const us_probe* probe, int32_t n_tx, int64_t ray_count,
                                  int32_t max_bounces);
int us_simulate_rf_recorded(us_ctx* ctx, us_scene* scene, const us_probe* probe, const us_tx_desc* tx,
                            int32_t n_tx, uint64_t seed, int32_t rays_per_elem, int64_t ray_begin,
                            int64_t ray_count, int32_t max_bounces, float* rf_dev, int64_t* counters_dev,
                            void* ws_dev, size_t ws_bytes, void* stream);
int us_simulate_rf_vjp_recorded(us_ctx* ctx, const us_scene* scene, const us_probe* probe, const us_tx_desc* tx,
                                int32_t n_tx, uint64_t seed, int32_t rays_per_elem, int64_t ray_begin,
                                int64_t ray_count, int32_t max_bounces, const float* g_rf_dev, double* g_theta_dev,
                                void* ws_dev, size_t ws_bytes, void* stream);
size_t us_frame_vjp_recorded_workspace_size(const us_probe* probe, const us_grid_desc* grid, int32_t n_tx);
int us_frame_vjp_recorded(us_ctx* ctx, const us_scene* scene, const us_probe* probe, const us_grid_desc* grid,
                          const us_tx_desc* tx, int32_t n_tx, uint64_t seed, int32_t rays_per_elem,
                          int64_t ray_begin, int64_t ray_count, int32_t max_bounces, const float* iq_dev,
                          const float* g_bmode_dev, float dr_db, double* g_theta_dev, void* ws_dev,
                          size_t ws_bytes, void* rec_dev, size_t rec_bytes, void* stream);

/* Inverse loop (Sec. "Parameterization and constraints", Sec. "Optimization
 * procedure", Algorithm opt). All arrays are device doubles of length n.
 *
 * us_param_map: theta[j] = lo[j] + clip(u[j], 0, 1) (hi[j] - lo[j])
 * (Eq. clip01, Eq. scale_phys); a parameter with lo[j] == hi[j] is fixed at
 * lo[j]. Requires lo[j] <= hi[j] (not checked on the device). */
int us_param_map(us_ctx* ctx, const double* u_dev, const double* lo_dev, const double* hi_dev,
                 int32_t n, double* theta_dev, void* stream);
/* us_adam_step: one Adam update (Eq. adam) of the unconstrained variables u
 * from the gradient with respect to theta (as accumulated by the VJPs):
 *   g_u[j] = g_theta[j] (hi[j] - lo[j]) if 0 < u[j] < 1 and lo[j] < hi[j],
 *            else 0                                       (Eq. clip_grad)
 *   if max_norm > 0 and |g_u|_2 > max_norm: g_u *= max_norm / |g_u|_2
 *   m = beta1 m + (1 - beta1) g_u;  v = beta2 v + (1 - beta2) g_u^2
 *   u -= lr[j] (m / (1 - beta1^step)) / (sqrt(v / (1 - beta2^step)) + eps)
 * step >= 1 counts the updates (bias correction); lr holds one learning rate
 * per parameter, so parameter groups are runs of equal values. u, m and v
 * are updated in place; m and v start at zero. */
int us_adam_step(us_ctx* ctx, double* u_dev, double* m_dev, double* v_dev,
                 const double* g_theta_dev, const double* lo_dev, const double* hi_dev,
                 const double* lr_dev, int32_t n, int32_t step, double beta1, double beta2,
                 double eps, double max_norm, void* stream);

/* Kernel timing for measurement. While enabled on a context, every kernel the
 * library launches for that context is bracketed by a pair of HIP events
 * recorded on the kernel's own stream. us_profile_read waits for the pending
 * events and returns, per kernel name, the summed duration in milliseconds and
 * the launch count, then clears the totals. names: caller buffer of
 * max_kernels * 32 chars (NUL-terminated names); *n_kernels receives the count
 * (kernels beyond max_kernels are dropped). Not thread-safe per context. */
int us_profile_enable(us_ctx* ctx, int enable);
int us_profile_read(us_ctx* ctx, int32_t max_kernels, char* names, double* total_ms,
                    int64_t* launches, int32_t* n_kernels);

#ifdef __cplusplus
}
#endif
#endif /* USRT_H */
