/*
 * pcgpu.h -- C ABI of the MI355X (gfx950) point-cloud hot path:
 * k-nearest-neighbour search, PCA normals and point-to-plane ICP.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Point sets are contiguous float32 arrays of n points with x, y, z
 *    consecutive: row-major (n, 3), which is byte-identical to the paper's
 *    one-point-per-column, column-major 3 x n view of contiguous data
 *    (Section 2, "Simple data representations").
 *  - Every array argument is a DEVICE pointer unless marked (host).  Arrays
 *    must be 4-byte aligned (8-byte for double), must not overlap an output
 *    unless stated, and stay owned by the caller: the library never
 *    allocates, frees or keeps device memory.  Scratch space comes from the
 *    caller's `workspace`, at least *_workspace_size() bytes, 256-byte
 *    aligned, whose contents are undefined on entry and on return.
 *  - All device work is enqueued on `stream` and is asynchronous; the host
 *    returns after argument validation and kernel launches.  Results are
 *    valid once the stream has reached the point of the call.
 *  - Errors: PC_EINVAL is returned synchronously, before any device work,
 *    for a null required pointer, a misaligned pointer, a size or parameter
 *    out of range; PC_EWORKSPACE when `workspace_bytes` is too small;
 *    PC_EDEVICE when a kernel launch fails.  No exception or abort crosses
 *    this interface.  Geometric outcomes of ICP (degenerate system, no
 *    inliers) are not errors; they are reported in pc_icp_stats.status.
 *  - Precondition: all coordinates and normals are finite.
 *  - Point counts must be below 2^31.
 */
#ifndef PCGPU_H
#define PCGPU_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PC_OK = 0,
    PC_EINVAL = 1,
    PC_EWORKSPACE = 2,
    PC_EDEVICE = 3
} pc_status;

enum {
    PC_ICP_CONVERGED = 0,   /* max |increment| fell below conv_tol        */
    PC_ICP_MAXITER = 1,     /* ran max_iters iterations                   */
    PC_ICP_DEGENERATE = 2,  /* fewer than 6 inliers or a singular 6x6 system */
    PC_ICP_NO_INLIERS = 3   /* no correspondence within max_corr_dist     */
};

enum { PCGPU_KMAX = 32 };   /* largest k for knn_search / estimate_normals */
/* Most clouds (pairs) in one batched call: the batch's search structure
 * sorts points by (cloud, Morton key) in 64-bit keys with 16 bits for the
 * cloud.  Batched calls and their workspace-size queries reject more (the
 * size queries return 0); icp_learned_batched replicates up to every pair
 * 8 times for its multi-start fallback, so it takes at most
 * PCGPU_MAX_CLOUDS / 8 pairs. */
enum { PCGPU_MAX_CLOUDS = 65536 };

/* Human-readable name of a status code (static string). */
const char *pc_status_string(pc_status s);

/* ------------------------------------------------------------------------
 * knn_search -- exact k nearest neighbours (Section 3, "Core operations":
 * k-NN queries of the KDTree).
 *
 * For each query q_i the k reference points with the smallest float32 key
 *     dx = r.x - q.x, dy = r.y - q.y, dz = r.z - q.z   (float32)
 *     key = fmaf(dz, dz, fmaf(dy, dy, dx * dx))
 * in ascending (key, reference index) order: ties go to the lower index.
 * A query that is also a reference point finds itself (key 0).
 *
 *   ref_xyz  (n_ref, 3) float32, n_ref >= 1
 *   qry_xyz  (n_qry, 3) float32, n_qry >= 0; may alias ref_xyz
 *   k        1 <= k <= min(n_ref, PCGPU_KMAX)
 *   out_idx  (n_qry, k) int32 reference indices, row i sorted as above
 *   out_d2   (n_qry, k) float32 keys, or NULL
 * ---------------------------------------------------------------------- */
size_t knn_search_workspace_size(int64_t n_ref, int64_t n_qry, int k);
pc_status knn_search(const float *ref_xyz, int64_t n_ref,
                     const float *qry_xyz, int64_t n_qry,
                     int k, int32_t *out_idx, float *out_d2,
                     void *workspace, size_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * estimate_normals -- PCA surface normals and curvature (Section 3, "Core
 * operations": normal and curvature estimation, PCA; Section 4: k-NN
 * neighbourhoods, viewpoint-consistent orientation).
 *
 * For each point p_i: N(i) = its k nearest points in the same cloud as
 * defined by knn_search (p_i included); C = (1/k) sum (x - mu)(x - mu)^T over
 * N(i); the normal is the unit eigenvector of C's smallest eigenvalue,
 * flipped so that n . (viewpoint - p_i) >= 0 (when that product is exactly
 * 0, the first nonzero component is made positive); curvature is the surface
 * variation l0 / (l0 + l1 + l2), 0 when the trace is 0.  A neighbourhood of
 * coincident points has normal (0, 0, 0) and curvature 0.
 *
 *   xyz            (n, 3) float32, n >= 0 (n == 0 is a no-op)
 *   k              1 <= k <= min(n, PCGPU_KMAX)
 *   viewpoint      (host) 3 floats
 *   out_normals    (n, 3) float32, in input order
 *   out_curvature  (n) float32, or NULL
 * ---------------------------------------------------------------------- */
size_t estimate_normals_workspace_size(int64_t n, int k);
pc_status estimate_normals(const float *xyz, int64_t n, int k, const float viewpoint[3],
                           float *out_normals, float *out_curvature,
                           void *workspace, size_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * estimate_normals_radius -- normals from radius neighbourhoods (Section 3,
 * "Core operations": radius and hybrid queries; Section 4: normals from the
 * points within 1 cm).
 *
 * k == 0: N(i) = every point with key(p_j, p_i) <= r2, where key is the
 * knn_search key and r2 = radius * radius rounded to float32 (so membership
 * is exact).  k > 0 (hybrid): the k nearest points of i with key <= r2.
 * Covariance, normal, orientation and curvature as in estimate_normals over
 * N(i); fewer than 3 points in N(i) give normal (0, 0, 0) and curvature 0.
 *   radius     finite, > 0
 *   k          0, or 1 <= k <= min(n, PCGPU_KMAX)
 * The workspace is estimate_normals_workspace_size(n, k).
 * ---------------------------------------------------------------------- */
pc_status estimate_normals_radius(const float *xyz, int64_t n, float radius, int k,
                                  const float viewpoint[3], float *out_normals, float *out_curvature,
                                  void *workspace, size_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * icp_point_to_plane -- rigid point-to-plane ICP (Section 3, "Iterative
 * geometric registration": alternate correspondence search and transform
 * estimation; the linear least-squares point-to-plane estimator of Low 2004
 * it cites; Section 4: nearest-neighbour correspondences with a rejection
 * distance and a fixed iteration count).
 *
 * T maps source to target (target ~ R * source + t), starting at init_T.
 * Each iteration: p'_i = R p_i + t, q_j = nearest target point of p'_i
 * (squared distance in float64, ties to the lower target index); the pair
 * is an inlier when |p'_i - q_j|^2 <= max_corr_dist^2 (float64) and
 * n_j != 0; r_i = (p'_i - q_j) . n_j, J_i = [p'_i x n_j, n_j];
 * x = -(sum J^T J)^{-1} sum J^T r = (alpha, beta, gamma, tau) solved in
 * float64 by Cholesky; R <- Rz(gamma) Ry(beta) Rx(alpha) R,
 * t <- Rz Ry Rx t + tau in float64.  The loop stops after max_iters
 * iterations, or earlier with PC_ICP_CONVERGED when conv_tol > 0 and
 * max |x_i| < conv_tol, or with PC_ICP_DEGENERATE / PC_ICP_NO_INLIERS
 * (fewer than 6 inliers or a Cholesky pivot <= 1e-14 * max diag; the pose
 * is then kept).  A last correspondence pass at the returned pose gives the
 * inlier count and rms = sqrt(sum r^2 / inliers).
 *
 *   src_xyz        (n_src, 3) float32, n_src >= 0
 *   tgt_xyz        (n_tgt, 3) float32, n_tgt >= 0
 *   tgt_normals    (n_tgt, 3) float32 target normals (e.g. estimate_normals)
 *   init_T         16 float64 row-major, or NULL for identity
 *   max_corr_dist  finite, > 0
 *   max_iters      >= 0
 *   conv_tol       finite, >= 0 (0 disables the early stop)
 *   out_T          16 float64 row-major (may alias init_T)
 *   out_stats      one pc_icp_stats (device), or NULL
 * When n_src or n_tgt is 0, out_T = init_T and status = PC_ICP_NO_INLIERS.
 *
 * On the device p'_i is formed in double-float arithmetic (float32 hi + lo
 * pairs of the float64 pose, about 2^-44 relative); the nearest point and
 * the d_max test are decided in float32 when an error bound proves the
 * float64 decision equal, and re-decided in float64 otherwise.  The sums are
 * compensated float32 (hi, lo) pairs merged in a fixed order, so the result
 * does not depend on scheduling.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t status;          /* PC_ICP_*                          */
    int32_t iterations_run;  /* increments applied                */
    int64_t inliers;         /* at the returned pose              */
    double rms;              /* sqrt(sum r^2 / inliers), 0 if none */
} pc_icp_stats;

size_t icp_point_to_plane_workspace_size(int64_t n_src, int64_t n_tgt, int max_iters);
pc_status icp_point_to_plane(const float *src_xyz, int64_t n_src,
                             const float *tgt_xyz, const float *tgt_normals, int64_t n_tgt,
                             const double *init_T, float max_corr_dist, int max_iters,
                             double conv_tol, double *out_T, pc_icp_stats *out_stats,
                             void *workspace, size_t workspace_bytes, hipStream_t stream);

/* icp_point_to_plane_noalloc -- icp_point_to_plane for callers that
 * cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, results
 * and kernels as icp_point_to_plane, without the workspace: the library
 * uses a device scratch array of PCGPU_NOALLOC_SCRATCH_BYTES that it holds
 * on each GPU it runs on from the first such call until the process ends.
 * The call itself allocates and frees nothing.
 *   Returns PC_EWORKSPACE, before any device work, when
 *   icp_point_to_plane_workspace_size(n_src, n_tgt, max_iters) exceeds
 *   PCGPU_NOALLOC_SCRATCH_BYTES (about 340,000 points per cloud at 30
 *   iterations); PC_EDEVICE when the scratch address cannot be obtained.
 * Every call on one GPU shares that GPU's scratch, and the scratch keeps the
 * last call's contents (each call initialises what it reads): calls that
 * overlap on one GPU (concurrent streams or threads) race and must be
 * serialised by the caller. */
#define PCGPU_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
pc_status icp_point_to_plane_noalloc(const float *src_xyz, int64_t n_src,
                                     const float *tgt_xyz, const float *tgt_normals, int64_t n_tgt,
                                     const double *init_T, float max_corr_dist, int max_iters,
                                     double conv_tol, double *out_T, pc_icp_stats *out_stats,
                                     hipStream_t stream);

/* icp_point_to_plane with the target normals estimated in the same call:
 * the target pyramid is built once and serves both the normals
 * (estimate_normals with k and viewpoint) and the correspondences.  The
 * result equals estimate_normals followed by icp_point_to_plane with those
 * normals, bit for bit.
 *   k            1 <= k <= min(n_tgt, PCGPU_KMAX)
 *   out_normals  (n_tgt, 3) float32 target normals, or NULL (then kept in
 *                the workspace only) */
size_t icp_point_to_plane_with_normals_workspace_size(int64_t n_src, int64_t n_tgt, int max_iters);
pc_status icp_point_to_plane_with_normals(const float *src_xyz, int64_t n_src,
                                          const float *tgt_xyz, int64_t n_tgt, int k,
                                          const float viewpoint[3], const double *init_T,
                                          float max_corr_dist, int max_iters, double conv_tol,
                                          double *out_T, pc_icp_stats *out_stats, float *out_normals,
                                          void *workspace, size_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Metric variants of the same loop (Section 3, "Iterative geometric
 * registration": point-to-point and point-to-plane metrics and weighted
 * combinations).  Correspondences, rejection, stopping rules, statuses and
 * the workspace (icp_point_to_plane_workspace_size) are those of
 * icp_point_to_plane.
 *
 * icp_point_to_point -- Besl and McKay (1992): each iteration fits the
 * least-squares rigid motion of the inlier pairs in closed form (centroids
 * and cross-covariance H = sum (p' - pbar)(q - qbar)^T; rotation by Horn's
 * 1987 unit-quaternion method, the same solution as Arun et al.'s SVD with
 * the reflection case excluded) and composes it on the left of the pose.
 * Fewer than 3 inliers, or a top-eigenvalue gap of Horn's matrix not above
 * 1e-6 times that eigenvalue (no unique rotation to that relative level,
 * e.g. nearly collinear pairs): PC_ICP_DEGENERATE.  Converged when max(|dR - I|, |dt|) < conv_tol.
 * rms = sqrt(sum |p' - q|^2 / inliers).  No normals are used.
 *
 * icp_combined -- the linearised least squares of
 *     w_plane * sum ((p' - q) . n)^2 + w_point * sum |p' - q|^2
 * under p' -> p' + omega x p' + tau: J_plane = [p' x n, n], J_point =
 * [-[p']_x, I]; A = w_plane J_plane^T J_plane + w_point J_point^T J_point,
 * b likewise, solved and applied as in icp_point_to_plane;
 * rms = sqrt(weighted sum / inliers).  w_point, w_plane finite, >= 0, not
 * both 0; tgt_normals may be NULL when w_plane is 0.  Weights (0, 1) give
 * icp_point_to_plane exactly.
 * ---------------------------------------------------------------------- */
pc_status icp_point_to_point(const float *src_xyz, int64_t n_src,
                             const float *tgt_xyz, int64_t n_tgt,
                             const double *init_T, float max_corr_dist, int max_iters,
                             double conv_tol, double *out_T, pc_icp_stats *out_stats,
                             void *workspace, size_t workspace_bytes, hipStream_t stream);
pc_status icp_combined(const float *src_xyz, int64_t n_src,
                       const float *tgt_xyz, const float *tgt_normals, int64_t n_tgt,
                       const double *init_T, float w_point, float w_plane,
                       float max_corr_dist, int max_iters, double conv_tol,
                       double *out_T, pc_icp_stats *out_stats,
                       void *workspace, size_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * icp_projective -- point-to-plane ICP with projective data association
 * (Section 3, "Iterative geometric registration": correspondences by
 * projective data association for the 3D case), for an organized target:
 * one point per pixel of a width x height image in raster order, taken by
 * a pinhole camera at the target frame's origin looking along +z.  A pixel
 * is valid when its point is finite with z > 0.  Each iteration, for
 * p' = T p in float64:
 *     u = fx * p'x / p'z + cx,  v = fy * p'y / p'z + cy   (float64, this order)
 *     pixel (floor(u + 0.5), floor(v + 0.5)) when p'z > 0 and inside the image;
 * the pair (p', q = that pixel's point) is an inlier when the pixel is valid,
 * its normal n != 0 and |p' - q|^2 <= max_corr_dist^2 (float64).  The
 * estimator, stopping rules and statistics are those of icp_point_to_plane.
 * No spatial index is built.
 *   tgt_xyz, tgt_normals   (height * width, 3) float32, organized
 *   intrinsics             (host) fx, fy (> 0), cx, cy
 * ---------------------------------------------------------------------- */
size_t icp_projective_workspace_size(int64_t n_src, int max_iters);
pc_status icp_projective(const float *src_xyz, int64_t n_src,
                         const float *tgt_xyz, const float *tgt_normals, int width, int height,
                         const float intrinsics[4], const double *init_T,
                         float max_corr_dist, int max_iters, double conv_tol,
                         double *out_T, pc_icp_stats *out_stats,
                         void *workspace, size_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Batched forms: many clouds or pairs of uneven sizes in one call, each
 * computed exactly as the single form would compute it alone.  Clouds are
 * packed back to back; offsets (host, m + 1 entries, offsets[0] = 0,
 * non-decreasing, total below 2^31) give cloud c as rows
 * [offsets[c], offsets[c+1]) of the packed array.  The offsets and the
 * per-item parameters travel to the device as kernel arguments of small
 * copy kernels launched by the call (so the host arrays may be freed on
 * return); everything else is asynchronous.  estimate_normals_batched,
 * icp_point_to_plane_batched and icp_point_to_plane_with_normals_batched
 * launch kernels only (no memset, no host copy): with the workspace and
 * outputs preallocated, a call can be captured in a graph and replayed.
 * ---------------------------------------------------------------------- */

/* estimate_normals on n_clouds clouds (neighbourhoods never cross clouds).
 *   xyz            (offsets[n_clouds], 3) float32, packed clouds
 *   offsets        (host) n_clouds + 1 int64
 *   k              (host) n_clouds int32, 1 <= k[c] <= min(n_c, PCGPU_KMAX)
 *                  (any value in range for an empty cloud)
 *   viewpoint      (host) 3 floats, shared by all clouds
 *   out_normals    (offsets[n_clouds], 3) float32, packed like xyz
 *   out_curvature  (offsets[n_clouds]) float32, or NULL */
size_t estimate_normals_batched_workspace_size(int n_clouds, const int64_t *offsets);
pc_status estimate_normals_batched(int n_clouds, const float *xyz, const int64_t *offsets,
                                   const int32_t *k, const float viewpoint[3],
                                   float *out_normals, float *out_curvature,
                                   void *workspace, size_t workspace_bytes, hipStream_t stream);

/* icp_point_to_plane on n_pairs independent pairs: pair p registers source
 * rows [src_off[p], src_off[p+1]) to target rows [tgt_off[p], tgt_off[p+1])
 * with its own pose, max_corr_dist[p] and max_iters[p]; conv_tol is shared.
 *   src_off, tgt_off   (host) n_pairs + 1 int64
 *   init_T             (n_pairs, 16) float64 row-major (device), or NULL
 *   max_corr_dist      (host) n_pairs float32, finite, > 0
 *   max_iters          (host) n_pairs int32, >= 0
 *   out_T              (n_pairs, 16) float64 (device)
 *   out_stats          n_pairs pc_icp_stats (device), or NULL
 * The workspace size takes the largest max_iters of the batch. */
size_t icp_point_to_plane_batched_workspace_size(int n_pairs, const int64_t *src_off,
                                                 const int64_t *tgt_off, int max_iters_max);
pc_status icp_point_to_plane_batched(int n_pairs, const float *src_xyz, const int64_t *src_off,
                                     const float *tgt_xyz, const float *tgt_normals,
                                     const int64_t *tgt_off, const double *init_T,
                                     const float *max_corr_dist, const int32_t *max_iters,
                                     double conv_tol, double *out_T, pc_icp_stats *out_stats,
                                     void *workspace, size_t workspace_bytes, hipStream_t stream);

/* icp_point_to_plane_with_normals on n_pairs independent pairs, packed as
 * in icp_point_to_plane_batched: the targets' normals (k[p] neighbours for
 * target p, host array; viewpoint shared) and the registrations share one
 * pyramid over all targets.  Each pair's pose, statistics and normals equal
 * those of icp_point_to_plane_with_normals on that pair alone.
 *   out_normals  (tgt_off[n_pairs], 3) float32 (device), or NULL */
size_t icp_point_to_plane_with_normals_batched_workspace_size(int n_pairs, const int64_t *src_off,
                                                              const int64_t *tgt_off, int max_iters_max);
pc_status icp_point_to_plane_with_normals_batched(int n_pairs, const float *src_xyz, const int64_t *src_off,
                                                  const float *tgt_xyz, const int64_t *tgt_off,
                                                  const int32_t *k, const float viewpoint[3],
                                                  const double *init_T, const float *max_corr_dist,
                                                  const int32_t *max_iters, double conv_tol, double *out_T,
                                                  pc_icp_stats *out_stats, float *out_normals,
                                                  void *workspace, size_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Learned pose initialiser and multi-start ICP.  Not part of the paper's
 * method, whose ICP starts from a given pose (Section 3, "Iterative
 * geometric registration"); these entry points supply that pose.
 *
 * Network (flat float32 parameters, pose_net_param_count() of them, in this
 * order, row-major W[in][out]): W1 3x64, b1 64, W2 64x128, b2 128, W3
 * 128x256, b3 256, W4 512x256, b4 256, W5 256x4, b5 4.  Per cloud, points
 * are centred on the centroid and scaled by the inverse RMS distance to it;
 * per point 3 -> 64 -> 128 -> 256 with ReLU after each layer, the inputs of
 * the second and third layers and W2, W3 rounded to bfloat16 (matrix cores,
 * float32 accumulation); the cloud feature f is the per-channel maximum.
 * Per pair: h = ReLU(W4^T [f_src; f_tgt] + b4), q = W5^T h + b5, R the
 * rotation of the unit quaternion q / |q| (w, x, y, z; the identity when
 * q = 0) and T0 = [R, c_tgt - R c_src] with c the centroids.  Pairs are
 * packed as in the batched forms (host offsets src_off, tgt_off).
 * ---------------------------------------------------------------------- */
int pose_net_param_count(void);
/* workspace of pose_net_predict and pose_net_train_step */
size_t pose_net_workspace_size(int n_pairs, const int64_t *src_off, const int64_t *tgt_off);
/* T0 of every pair into out_T (n_pairs, 16) float64. */
pc_status pose_net_predict(const float *params, int n_pairs,
                           const float *src_xyz, const int64_t *src_off,
                           const float *tgt_xyz, const int64_t *tgt_off,
                           double *out_T, void *workspace, size_t workspace_bytes,
                           hipStream_t stream);
/* One training step on n_pairs pairs with label poses label_T (n_pairs,
 * 16; only the rotation is used): loss_p = w_p |R_p - R_label,p|_F^2 with
 * w_p = pair_weight[p] (NULL: all 1).  The gradient of sum_p loss_p is taken
 * with the bfloat16 roundings passed through unchanged; when lr > 0, Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected with `step` >= 1)
 * updates params in place with that gradient divided by sum_p w_p, using
 * and updating the caller's moment arrays adam_m, adam_v (pose_net_param_count
 * floats each, zero before step 1).  lr = 0 leaves params, adam_m and adam_v
 * untouched (they may be NULL).  Optional outputs: out_loss (n_pairs
 * float32, loss_p), out_grad (pose_net_param_count float32, the summed
 * gradient).  Deterministic: no atomics. */
pc_status pose_net_train_step(float *params, float *adam_m, float *adam_v, int step, float lr,
                              int n_pairs, const float *src_xyz, const int64_t *src_off,
                              const float *tgt_xyz, const int64_t *tgt_off,
                              const double *label_T, const float *pair_weight,
                              float *out_loss, float *out_grad,
                              void *workspace, size_t workspace_bytes, hipStream_t stream);

/* Registration of n_pairs packed pairs by icp_point_to_plane_batched
 * (shared max_corr_dist and max_iters) from:
 *   PC_INIT_LEARNED       T0 of the network; pairs whose result is not
 *                         (status CONVERGED or MAXITER, inliers > 0 and
 *                         rms <= accept_rms) are registered again by
 *                         multi-start ICP and take its result;
 *   PC_INIT_MULTI_START   multi-start ICP for every pair (params unused,
 *                         may be NULL);
 *   PC_INIT_LEARNED_ONLY  T0 of the network, no fallback.
 * Multi-start ICP runs kStarts = 8 registrations per pair, from the
 * rotations identity and 60 degrees about each of the 7 Fibonacci-sphere
 * axes a_i = (r cos(i g), r sin(i g), z), z = 1 - (2i + 1) / 7,
 * r = sqrt(1 - z^2), g = pi (3 - sqrt 5), each about the source centroid
 * onto the target centroid, and keeps the first start unless a later one
 * has inliers and either the kept one has none or a lower rms.
 *   out_T      (n_pairs, 16) float64
 *   out_stats  n_pairs pc_icp_stats, or NULL
 *   out_start  n_pairs int32 (device), or NULL: -1 when the learned start
 *              was kept, else the multi-start index 0..7
 * With PC_INIT_LEARNED the call waits for the stream once (the fallback
 * set depends on the first results).  Points per side times 8 must stay
 * below 2^31. */
enum { PC_INIT_LEARNED = 0, PC_INIT_MULTI_START = 1, PC_INIT_LEARNED_ONLY = 2 };
size_t icp_learned_batched_workspace_size(int n_pairs, const int64_t *src_off, const int64_t *tgt_off,
                                          int max_iters);
pc_status icp_learned_batched(int mode, const float *params, int n_pairs,
                              const float *src_xyz, const int64_t *src_off,
                              const float *tgt_xyz, const float *tgt_normals, const int64_t *tgt_off,
                              float max_corr_dist, int max_iters, double conv_tol, float accept_rms,
                              double *out_T, pc_icp_stats *out_stats, int32_t *out_start,
                              void *workspace, size_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Tuning (process-wide; not thread-safe): launch shape and pyramid depth of
 * later calls.  Every setting finds the same exact neighbours and
 * correspondences; the block size only regroups the compensated per-block
 * sums, which moves them by about 1e-14 relative.  Workspace sizes do not
 * depend on the tuning.
 *   icp_block_threads  64, 128 or 256: source points per accumulate block
 *   icp_leaf           8, 16 or 32: nodes holding at most this many points
 *                      are scanned whole by the searches (ICP
 *                      correspondences, k-NN, normals)
 *   node_budget        0.125 .. 1: the finest pyramid level of a cloud is
 *                      the finest one whose levels hold at most
 *                      node_budget * n nodes (smaller: coarser leaves); used
 *                      by estimate_normals* and icp_point_to_plane*
 *   sort_queries       0 or 1: ICP with nearest-neighbour correspondences
 *                      visits the source points of each pair in the Morton
 *                      order of their own cube (sorted once per call) rather
 *                      than in input order, so neighbouring lanes search
 *                      neighbouring cells; pays off when the input order is
 *                      not already spatially coherent.  Changes only the
 *                      order of the compensated sums.
 *   icp_persistent     must be 0.  Reserved for running the whole
 *                      point-to-plane loop as one cooperative launch of
 *                      co-resident workgroups with grid barriers between
 *                      its phases; that form is switched off (a run of it
 *                      stopped making progress and the cause is not
 *                      established), so pc_set_tuning rejects 1.
 * Defaults: 128, 16, 1, 1, 0.  pc_set_tuning returns PC_EINVAL for other
 * values.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t icp_block_threads;
    int32_t icp_leaf;
    float node_budget;
    int32_t sort_queries;
    int32_t icp_persistent;
} pc_tuning;

pc_status pc_set_tuning(const pc_tuning *t);
void pc_get_tuning(pc_tuning *t);

/* ------------------------------------------------------------------------
 * Diagnostics
 * ---------------------------------------------------------------------- */
/* Streams n_bytes (multiple of 16) from src to dst with one read and one
   write per byte; used to calibrate bandwidth and hardware counters. */
pc_status pc_copy_probe(void *dst, const void *src, size_t n_bytes, hipStream_t stream);

/* Per-iteration history of the last icp_point_to_plane call that used this
   workspace: for iteration i, 8 float64 values (alpha, beta, gamma, tau_x,
   tau_y, tau_z, inliers, sum r^2) at the pose before the increment.  Returns
   a device pointer into `workspace` (valid until it is reused), or NULL. */
const double *icp_history(void *workspace, size_t workspace_bytes,
                          int64_t n_src, int64_t n_tgt, int max_iters);

/* Registers caller-owned HIP events (created with timing enabled) that
   icp_point_to_plane and icp_point_to_plane_batched record on their stream
   immediately before and after the correspondence/accumulation kernel of
   iteration i, for i < capacity; knn_search and estimate_normals record
   slot 0 around their search kernel (k_knn, k_normals); pose_net_predict
   records slot 0 around the encoder kernel; pose_net_train_step
   records slot 0 around the forward, 1 around the backward and 2 around
   the second-layer weight-gradient kernel.  Pass
   capacity 0 to stop.  pc_kernel_timer_count() returns how many pairs the
   last call recorded.  For measurement only; not thread-safe. */
pc_status pc_set_kernel_timer(hipEvent_t *begin, hipEvent_t *end, int capacity);
int pc_kernel_timer_count(void);

#ifdef __cplusplus
}
#endif

#endif /* PCGPU_H */
