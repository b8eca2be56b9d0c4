// C-ABI entry points: argument validation, workspace carving, launches.

#include <math.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "icp.h"
#include "pose_net.h"

using namespace pcg;

namespace {

constexpr int64_t kMaxPoints = (int64_t)1 << 31;

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

// host offsets of m items (1 <= m <= max_m; batches of clouds are limited by
// the cloud bits of the sort keys): off[0] = 0, non-decreasing, total below
// kMaxPoints
bool valid_offsets(const int64_t *off, int m, int max_m = PCGPU_MAX_CLOUDS)
{
    if (!off || m < 1 || m > max_m || off[0] != 0) return false;
    for (int i = 0; i < m; i++)
        if (off[i + 1] < off[i]) return false;
    return off[m] < kMaxPoints;
}

// process-wide tuning of the ICP kernels and the pyramid (pc_set_tuning)
pc_tuning g_tune = {128, 16, 1.0f, 1, 0};

// Small host arrays (offsets, per-pair parameters) reach the device as
// kernel arguments, kUploadChunk bytes per launch, copied by value when the
// kernel is launched.  A call then launches kernels only, so it can be
// captured in a graph (a copy from pageable host memory is not a safe graph
// node), and the caller's arrays need not outlive the call.  Every array
// uploaded holds 4- or 8-byte elements, at 4-byte aligned destinations.
constexpr int kUploadChunk = 2048;
struct UploadChunk {
    uint32_t w[kUploadChunk / 4];
};

__global__ void k_upload(UploadChunk c, uint32_t *__restrict__ dst, uint32_t nwords)
{
    for (uint32_t i = threadIdx.x; i < nwords; i += blockDim.x) dst[i] = c.w[i];
}

bool upload(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    if (bytes % 4 != 0 || ((uintptr_t)dst % 4) != 0) return false;
    for (size_t off = 0; off < bytes; off += kUploadChunk) {
        const size_t nb = bytes - off < (size_t)kUploadChunk ? bytes - off : (size_t)kUploadChunk;
        UploadChunk c;
        memcpy(c.w, static_cast<const char *>(src) + off, nb);
        k_upload<<<1, 256, 0, s>>>(c, reinterpret_cast<uint32_t *>(static_cast<char *>(dst) + off),
                                   (uint32_t)(nb / 4));
        if (hipGetLastError() != hipSuccess) return false;
    }
    return true;
}

__global__ void k_copy16(const uint4 *__restrict__ src, uint4 *__restrict__ dst, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// Scratch of icp_point_to_plane_noalloc: a file-scope device array, one
// copy per GPU, resident from the code object's load until the process
// ends.  Host code never uses its name as an address (on the host it is a
// stand-in symbol); the device address of the current GPU's copy comes from
// hipGetSymbolAddress, taken once per device with that device current.
__device__ __align__(256) unsigned char scratch[PCGPU_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// the current device's scratch address, or nullptr when it cannot be had
void *noalloc_scratch()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

const char *pc_status_string(pc_status s)
{
    switch (s) {
    case PC_OK: return "PC_OK";
    case PC_EINVAL: return "PC_EINVAL: invalid argument";
    case PC_EWORKSPACE: return "PC_EWORKSPACE: workspace too small";
    case PC_EDEVICE: return "PC_EDEVICE: device launch failed";
    }
    return "unknown pc_status";
}

size_t knn_search_workspace_size(int64_t n_ref, int64_t n_qry, int k)
{
    (void)n_qry;
    (void)k;
    if (n_ref < 0 || n_ref >= kMaxPoints) return 0;
    return grid_bytes(n_ref, 1);
}

pc_status knn_search(const float *ref_xyz, int64_t n_ref, const float *qry_xyz, int64_t n_qry, int k,
                     int32_t *out_idx, float *out_d2, void *workspace, size_t workspace_bytes, hipStream_t stream)
{
    if (n_ref < 1 || n_ref >= kMaxPoints || n_qry < 0 || n_qry >= kMaxPoints) return PC_EINVAL;
    if (k < 1 || k > PCGPU_KMAX || k > n_ref) return PC_EINVAL;
    if (!ref_xyz || !workspace || (n_qry > 0 && (!qry_xyz || !out_idx))) return PC_EINVAL;
    if (!aligned(ref_xyz, 4) || !aligned(qry_xyz, 4) || !aligned(out_idx, 4) || !aligned(out_d2, 4) ||
        !aligned(workspace, 256))
        return PC_EINVAL;
    if (workspace_bytes < knn_search_workspace_size(n_ref, n_qry, k)) return PC_EWORKSPACE;
    Carver c(workspace, workspace_bytes);
    GridStore g;
    grid_carve(c, n_ref, 1, g);
    if (!c.ok) return PC_EWORKSPACE;
    g.leaf = g_tune.icp_leaf;
    if (grid_set_single_cloud(g, stream) != hipSuccess) return PC_EDEVICE;
    if (grid_build(g, ref_xyz, stream) != hipSuccess) return PC_EDEVICE;
    if (knn_run(g, qry_xyz, n_qry, k, out_idx, out_d2, stream) != hipSuccess) return PC_EDEVICE;
    return PC_OK;
}

size_t estimate_normals_workspace_size(int64_t n, int k)
{
    (void)k;
    if (n < 0 || n >= kMaxPoints) return 0;
    return grid_bytes(n, 1);
}

pc_status estimate_normals(const float *xyz, int64_t n, int k, const float viewpoint[3], float *out_normals,
                           float *out_curvature, void *workspace, size_t workspace_bytes, hipStream_t stream)
{
    if (n < 0 || n >= kMaxPoints || !viewpoint) return PC_EINVAL;
    if (k < 1 || k > PCGPU_KMAX) return PC_EINVAL;
    if (n == 0) return PC_OK;
    if (k > n) return PC_EINVAL;
    if (!xyz || !out_normals || !workspace) return PC_EINVAL;
    if (!isfinite(viewpoint[0]) || !isfinite(viewpoint[1]) || !isfinite(viewpoint[2])) return PC_EINVAL;
    if (!aligned(xyz, 4) || !aligned(out_normals, 4) || !aligned(out_curvature, 4) || !aligned(workspace, 256))
        return PC_EINVAL;
    if (workspace_bytes < estimate_normals_workspace_size(n, k)) return PC_EWORKSPACE;
    Carver c(workspace, workspace_bytes);
    GridStore g;
    grid_carve(c, n, 1, g);
    if (!c.ok) return PC_EWORKSPACE;
    g.node_budget = g_tune.node_budget;
    g.leaf = g_tune.icp_leaf;
    if (grid_set_single_cloud(g, stream) != hipSuccess) return PC_EDEVICE;
    if (grid_build(g, xyz, stream) != hipSuccess) return PC_EDEVICE;
    if (normals_run(g, xyz, k, nullptr, viewpoint, out_normals, out_curvature, stream) != hipSuccess)
        return PC_EDEVICE;
    return PC_OK;
}

namespace {

// the batched normals carve: the grid, then the per-cloud k
int32_t *carve_normals_batched(Carver &c, int n_clouds, const int64_t *offsets, GridStore &g)
{
    grid_carve(c, offsets[n_clouds], n_clouds, g);
    return c.take<int32_t>(n_clouds);
}

}  // namespace

pc_status estimate_normals_radius(const float *xyz, int64_t n, float radius, int k, const float viewpoint[3],
                                  float *out_normals, float *out_curvature, void *workspace, size_t workspace_bytes,
                                  hipStream_t stream)
{
    if (n < 0 || n >= kMaxPoints || !viewpoint) return PC_EINVAL;
    if (!(radius > 0.f) || !isfinite(radius) || k < 0 || k > PCGPU_KMAX) return PC_EINVAL;
    if (!isfinite(viewpoint[0]) || !isfinite(viewpoint[1]) || !isfinite(viewpoint[2])) return PC_EINVAL;
    if (n == 0) return PC_OK;
    if (k > n) return PC_EINVAL;
    if (!xyz || !out_normals || !workspace) return PC_EINVAL;
    if (!aligned(xyz, 4) || !aligned(out_normals, 4) || !aligned(out_curvature, 4) || !aligned(workspace, 256))
        return PC_EINVAL;
    if (workspace_bytes < estimate_normals_workspace_size(n, k)) return PC_EWORKSPACE;
    Carver c(workspace, workspace_bytes);
    GridStore g;
    grid_carve(c, n, 1, g);
    if (!c.ok) return PC_EWORKSPACE;
    g.node_budget = g_tune.node_budget;
    g.leaf = g_tune.icp_leaf;
    if (grid_set_single_cloud(g, stream) != hipSuccess) return PC_EDEVICE;
    if (grid_build(g, xyz, stream) != hipSuccess) return PC_EDEVICE;
    const float r2 = radius * radius;
    hipError_t e = k == 0 ? normals_radius_run(g, r2, viewpoint, out_normals, out_curvature, stream)
                          : normals_run(g, xyz, k, nullptr, viewpoint, out_normals, out_curvature, stream, r2, 3);
    return e == hipSuccess ? PC_OK : PC_EDEVICE;
}

size_t estimate_normals_batched_workspace_size(int n_clouds, const int64_t *offsets)
{
    if (n_clouds < 1 || !valid_offsets(offsets, n_clouds)) return 0;
    Carver c(nullptr, ~(size_t)0 >> 1);
    GridStore g;
    carve_normals_batched(c, n_clouds, offsets, g);
    return c.used();
}

pc_status estimate_normals_batched(int n_clouds, const float *xyz, const int64_t *offsets, const int32_t *k,
                                   const float viewpoint[3], float *out_normals, float *out_curvature,
                                   void *workspace, size_t workspace_bytes, hipStream_t stream)
{
    if (n_clouds < 1 || !valid_offsets(offsets, n_clouds) || !k || !viewpoint) return PC_EINVAL;
    const int64_t n = offsets[n_clouds];
    int k_max = 1;
    for (int c = 0; c < n_clouds; c++) {
        int64_t nc = offsets[c + 1] - offsets[c];
        if (k[c] < 1 || k[c] > PCGPU_KMAX || (nc > 0 && k[c] > nc)) return PC_EINVAL;
        k_max = k[c] > k_max ? k[c] : k_max;
    }
    if (!isfinite(viewpoint[0]) || !isfinite(viewpoint[1]) || !isfinite(viewpoint[2])) return PC_EINVAL;
    if (n == 0) return PC_OK;
    if (!xyz || !out_normals || !workspace) return PC_EINVAL;
    if (!aligned(xyz, 4) || !aligned(out_normals, 4) || !aligned(out_curvature, 4) || !aligned(workspace, 256))
        return PC_EINVAL;
    if (workspace_bytes < estimate_normals_batched_workspace_size(n_clouds, offsets)) return PC_EWORKSPACE;
    Carver c(workspace, workspace_bytes);
    GridStore g;
    int32_t *kc = carve_normals_batched(c, n_clouds, offsets, g);
    if (!c.ok) return PC_EWORKSPACE;
    g.node_budget = g_tune.node_budget;
    g.leaf = g_tune.icp_leaf;
    if (!upload(g.off, offsets, sizeof(int64_t) * (n_clouds + 1), stream)) return PC_EDEVICE;
    if (!upload(kc, k, sizeof(int32_t) * n_clouds, stream)) return PC_EDEVICE;
    if (grid_build(g, xyz, stream) != hipSuccess) return PC_EDEVICE;
    if (normals_run(g, xyz, k_max, kc, viewpoint, out_normals, out_curvature, stream) != hipSuccess)
        return PC_EDEVICE;
    return PC_OK;
}

namespace {

// The workspace layout does not depend on the tuning: block partials are
// carved for the smallest block size.  The launch shape is set afterwards.
void tune(IcpStore &s)
{
    s.threads = g_tune.icp_block_threads;
    s.leaf = g_tune.icp_leaf;
    s.grid.node_budget = g_tune.node_budget;
    s.grid.leaf = g_tune.icp_leaf;
    s.sort_src = g_tune.sort_queries != 0;
    s.persistent = g_tune.icp_persistent != 0;
}

// the single-pair carve, shared by the size query, the call and the history
void carve_single(Carver &c, int64_t n_src, int64_t n_tgt, int max_iters, IcpStore &s)
{
    int64_t cap = icp_blocks_max(n_src);
    icp_carve(c, 1, n_src, n_tgt, cap, icp_groups(cap), max_iters, s);
    tune(s);
    s.nblk = (int)icp_blocks(n_src, s.threads);
    s.ngrp = (int)icp_groups(s.nblk);
    s.max_pair_groups = s.ngrp;
}

// the batched carve: blocks and groups per pair from the host offsets
void carve_batched(Carver &c, int n_pairs, const int64_t *src_off, const int64_t *tgt_off, int iters_max,
                   IcpStore &s, std::vector<int32_t> *boff, std::vector<int32_t> *goff)
{
    int64_t cap_b = 0, cap_g = 0, nblk = 0, ngrp = 0, max_g = 0;
    const int threads = g_tune.icp_block_threads;
    if (boff) boff->assign(1, 0);
    if (goff) goff->assign(1, 0);
    for (int p = 0; p < n_pairs; p++) {
        int64_t ns = src_off[p + 1] - src_off[p];
        cap_b += icp_blocks_max(ns);
        cap_g += icp_groups(icp_blocks_max(ns));
        int64_t b = icp_blocks(ns, threads);
        nblk += b;
        ngrp += icp_groups(b);
        max_g = icp_groups(b) > max_g ? icp_groups(b) : max_g;
        if (boff) boff->push_back((int32_t)nblk);
        if (goff) goff->push_back((int32_t)ngrp);
    }
    icp_carve(c, n_pairs, src_off[n_pairs], tgt_off[n_pairs], cap_b, cap_g, iters_max, s);
    tune(s);
    s.nblk = (int)nblk;
    s.ngrp = (int)ngrp;
    s.max_pair_groups = (int)max_g;
}

}  // namespace

size_t icp_point_to_plane_workspace_size(int64_t n_src, int64_t n_tgt, int max_iters)
{
    if (n_src < 0 || n_tgt < 0 || n_src >= kMaxPoints || n_tgt >= kMaxPoints || max_iters < 0) return 0;
    Carver c(nullptr, ~(size_t)0 >> 1);
    IcpStore s;
    carve_single(c, n_src, n_tgt, max_iters, s);
    return c.used();
}

namespace {

// the single-pair ICP arguments other than the workspace (host only)
bool icp_single_args_ok(const float *src_xyz, int64_t n_src, const float *tgt_xyz, const float *tgt_normals,
                        int64_t n_tgt, const double *init_T, float max_corr_dist, int max_iters, double conv_tol,
                        const double *out_T, const pc_icp_stats *out_stats, bool need_normals)
{
    if (n_src < 0 || n_tgt < 0 || n_src >= kMaxPoints || n_tgt >= kMaxPoints) return false;
    if (max_iters < 0 || !(max_corr_dist > 0.f) || !isfinite(max_corr_dist)) return false;
    if (!(conv_tol >= 0.0) || !isfinite(conv_tol)) return false;
    if (!out_T) return false;
    if ((n_src > 0 && !src_xyz) || (n_tgt > 0 && (!tgt_xyz || (need_normals && !tgt_normals)))) return false;
    return aligned(src_xyz, 4) && aligned(tgt_xyz, 4) && aligned(tgt_normals, 4) && aligned(init_T, 8) &&
           aligned(out_T, 8) && aligned(out_stats, 8);
}

// single-pair ICP with any metric (0 point-to-plane, 1 point-to-point, 2 combined)
pc_status icp_single(const float *src_xyz, int64_t n_src, const float *tgt_xyz, const float *tgt_normals,
                     int64_t n_tgt, const double *init_T, float max_corr_dist, int max_iters, double conv_tol,
                     double *out_T, pc_icp_stats *out_stats, void *workspace, size_t workspace_bytes,
                     hipStream_t stream, int metric, float w_point, float w_plane)
{
    const bool need_normals = metric == 0 || (metric == 2 && w_plane > 0.f);
    if (!icp_single_args_ok(src_xyz, n_src, tgt_xyz, tgt_normals, n_tgt, init_T, max_corr_dist, max_iters,
                            conv_tol, out_T, out_stats, need_normals))
        return PC_EINVAL;
    if (!workspace || !aligned(workspace, 256)) return PC_EINVAL;
    if (workspace_bytes < icp_point_to_plane_workspace_size(n_src, n_tgt, max_iters)) return PC_EWORKSPACE;
    Carver c(workspace, workspace_bytes);
    IcpStore s;
    carve_single(c, n_src, n_tgt, max_iters, s);
    if (!c.ok) return PC_EWORKSPACE;
    s.metric = metric;
    s.w_point = w_point;
    s.w_plane = w_plane;
    if (icp_layout_single(s, n_src, n_tgt, max_corr_dist, max_iters, stream) != hipSuccess) return PC_EDEVICE;
    hipError_t e = icp_run(s, src_xyz, n_src, tgt_xyz, need_normals ? tgt_normals : nullptr, init_T, conv_tol,
                           out_T, out_stats, stream);
    return e == hipSuccess ? PC_OK : PC_EDEVICE;
}

}  // namespace

pc_status icp_point_to_plane(const float *src_xyz, int64_t n_src, const float *tgt_xyz, const float *tgt_normals,
                             int64_t n_tgt, const double *init_T, float max_corr_dist, int max_iters,
                             double conv_tol, double *out_T, pc_icp_stats *out_stats, void *workspace,
                             size_t workspace_bytes, hipStream_t stream)
{
    return icp_single(src_xyz, n_src, tgt_xyz, tgt_normals, n_tgt, init_T, max_corr_dist, max_iters, conv_tol,
                      out_T, out_stats, workspace, workspace_bytes, stream, 0, 0.f, 1.f);
}

pc_status icp_point_to_plane_noalloc(const float *src_xyz, int64_t n_src, const float *tgt_xyz,
                                     const float *tgt_normals, int64_t n_tgt, const double *init_T,
                                     float max_corr_dist, int max_iters, double conv_tol, double *out_T,
                                     pc_icp_stats *out_stats, hipStream_t stream)
{
    // every check on the host first: a rejected call does no device work
    if (!icp_single_args_ok(src_xyz, n_src, tgt_xyz, tgt_normals, n_tgt, init_T, max_corr_dist, max_iters,
                            conv_tol, out_T, out_stats, true))
        return PC_EINVAL;
    if (icp_point_to_plane_workspace_size(n_src, n_tgt, max_iters) > PCGPU_NOALLOC_SCRATCH_BYTES)
        return PC_EWORKSPACE;
    void *ws = noalloc_scratch();
    if (!ws) return PC_EDEVICE;
    return icp_single(src_xyz, n_src, tgt_xyz, tgt_normals, n_tgt, init_T, max_corr_dist, max_iters, conv_tol,
                      out_T, out_stats, ws, PCGPU_NOALLOC_SCRATCH_BYTES, stream, 0, 0.f, 1.f);
}

size_t icp_point_to_plane_with_normals_workspace_size(int64_t n_src, int64_t n_tgt, int max_iters)
{
    if (n_src < 0 || n_tgt < 0 || n_src >= kMaxPoints || n_tgt >= kMaxPoints || max_iters < 0) return 0;
    Carver c(nullptr, ~(size_t)0 >> 1);
    IcpStore s;
    carve_single(c, n_src, n_tgt, max_iters, s);
    c.take<float>((size_t)3 * (n_tgt > 0 ? n_tgt : 1));
    return c.used();
}

pc_status icp_point_to_plane_with_normals(const float *src_xyz, int64_t n_src, const float *tgt_xyz, int64_t n_tgt,
                                          int k, const float viewpoint[3], const double *init_T, float max_corr_dist,
                                          int max_iters, double conv_tol, double *out_T, pc_icp_stats *out_stats,
                                          float *out_normals, void *workspace, size_t workspace_bytes,
                                          hipStream_t stream)
{
    if (n_src < 0 || n_tgt < 0 || n_src >= kMaxPoints || n_tgt >= kMaxPoints || !viewpoint) return PC_EINVAL;
    if (k < 1 || k > PCGPU_KMAX || (n_tgt > 0 && k > n_tgt)) return PC_EINVAL;
    if (!isfinite(viewpoint[0]) || !isfinite(viewpoint[1]) || !isfinite(viewpoint[2])) return PC_EINVAL;
    if (max_iters < 0 || !(max_corr_dist > 0.f) || !isfinite(max_corr_dist)) return PC_EINVAL;
    if (!(conv_tol >= 0.0) || !isfinite(conv_tol)) return PC_EINVAL;
    if (!out_T || !workspace) return PC_EINVAL;
    if ((n_src > 0 && !src_xyz) || (n_tgt > 0 && !tgt_xyz)) return PC_EINVAL;
    if (!aligned(src_xyz, 4) || !aligned(tgt_xyz, 4) || !aligned(out_normals, 4) || !aligned(init_T, 8) ||
        !aligned(out_T, 8) || !aligned(out_stats, 8) || !aligned(workspace, 256))
        return PC_EINVAL;
    if (workspace_bytes < icp_point_to_plane_with_normals_workspace_size(n_src, n_tgt, max_iters))
        return PC_EWORKSPACE;
    Carver c(workspace, workspace_bytes);
    IcpStore s;
    carve_single(c, n_src, n_tgt, max_iters, s);
    float *nb = c.take<float>((size_t)3 * (n_tgt > 0 ? n_tgt : 1));
    if (!c.ok) return PC_EWORKSPACE;
    if (out_normals) nb = out_normals;
    if (icp_layout_single(s, n_src, n_tgt, max_corr_dist, max_iters, stream) != hipSuccess) return PC_EDEVICE;
    // one pyramid over the target serves its normals and the correspondences
    if (grid_build(s.grid, tgt_xyz, stream) != hipSuccess) return PC_EDEVICE;
    if (n_tgt > 0 &&
        normals_run(s.grid, tgt_xyz, k, nullptr, viewpoint, nb, nullptr, stream, INFINITY, 0, s.nrm) != hipSuccess)
        return PC_EDEVICE;
    s.grid_built = true;
    s.nrm_ready = true;
    hipError_t e = icp_run(s, src_xyz, n_src, tgt_xyz, nb, init_T, conv_tol, out_T, out_stats, stream);
    return e == hipSuccess ? PC_OK : PC_EDEVICE;
}

pc_status icp_point_to_point(const float *src_xyz, int64_t n_src, const float *tgt_xyz, int64_t n_tgt,
                             const double *init_T, float max_corr_dist, int max_iters, double conv_tol,
                             double *out_T, pc_icp_stats *out_stats, void *workspace, size_t workspace_bytes,
                             hipStream_t stream)
{
    return icp_single(src_xyz, n_src, tgt_xyz, nullptr, n_tgt, init_T, max_corr_dist, max_iters, conv_tol, out_T,
                      out_stats, workspace, workspace_bytes, stream, 1, 1.f, 0.f);
}

pc_status icp_combined(const float *src_xyz, int64_t n_src, const float *tgt_xyz, const float *tgt_normals,
                       int64_t n_tgt, const double *init_T, float w_point, float w_plane, float max_corr_dist,
                       int max_iters, double conv_tol, double *out_T, pc_icp_stats *out_stats, void *workspace,
                       size_t workspace_bytes, hipStream_t stream)
{
    if (!(w_point >= 0.f) || !(w_plane >= 0.f) || !isfinite(w_point) || !isfinite(w_plane) ||
        !(w_point + w_plane > 0.f))
        return PC_EINVAL;
    return icp_single(src_xyz, n_src, tgt_xyz, tgt_normals, n_tgt, init_T, max_corr_dist, max_iters, conv_tol,
                      out_T, out_stats, workspace, workspace_bytes, stream, 2, w_point, w_plane);
}

size_t icp_projective_workspace_size(int64_t n_src, int max_iters)
{
    if (n_src < 0 || n_src >= kMaxPoints || max_iters < 0) return 0;
    Carver c(nullptr, ~(size_t)0 >> 1);
    IcpStore s;
    carve_single(c, n_src, 0, max_iters, s);
    return c.used();
}

pc_status icp_projective(const float *src_xyz, int64_t n_src, const float *tgt_xyz, const float *tgt_normals,
                         int width, int height, const float intrinsics[4], const double *init_T,
                         float max_corr_dist, int max_iters, double conv_tol, double *out_T,
                         pc_icp_stats *out_stats, void *workspace, size_t workspace_bytes, hipStream_t stream)
{
    if (n_src < 0 || n_src >= kMaxPoints || width < 1 || height < 1 || !intrinsics) return PC_EINVAL;
    if ((int64_t)width * height >= kMaxPoints) return PC_EINVAL;
    for (int i = 0; i < 4; i++)
        if (!isfinite(intrinsics[i])) return PC_EINVAL;
    if (!(intrinsics[0] > 0.f) || !(intrinsics[1] > 0.f)) return PC_EINVAL;
    if (max_iters < 0 || !(max_corr_dist > 0.f) || !isfinite(max_corr_dist)) return PC_EINVAL;
    if (!(conv_tol >= 0.0) || !isfinite(conv_tol)) return PC_EINVAL;
    if (!out_T || !workspace || !tgt_xyz || !tgt_normals || (n_src > 0 && !src_xyz)) return PC_EINVAL;
    if (!aligned(src_xyz, 4) || !aligned(tgt_xyz, 4) || !aligned(tgt_normals, 4) || !aligned(init_T, 8) ||
        !aligned(out_T, 8) || !aligned(out_stats, 8) || !aligned(workspace, 256))
        return PC_EINVAL;
    if (workspace_bytes < icp_projective_workspace_size(n_src, max_iters)) return PC_EWORKSPACE;
    Carver c(workspace, workspace_bytes);
    IcpStore s;
    carve_single(c, n_src, 0, max_iters, s);
    if (!c.ok) return PC_EWORKSPACE;
    s.assoc = kAssocProjective;
    s.width = width;
    s.height = height;
    for (int i = 0; i < 4; i++) s.K[i] = intrinsics[i];
    const int64_t npix = (int64_t)width * height;
    if (icp_layout_single(s, n_src, npix, max_corr_dist, max_iters, stream) != hipSuccess) return PC_EDEVICE;
    hipError_t e = icp_run(s, src_xyz, n_src, tgt_xyz, tgt_normals, init_T, conv_tol, out_T, out_stats, stream);
    return e == hipSuccess ? PC_OK : PC_EDEVICE;
}

size_t icp_point_to_plane_batched_workspace_size(int n_pairs, const int64_t *src_off, const int64_t *tgt_off,
                                                 int max_iters_max)
{
    if (n_pairs < 1 || max_iters_max < 0 || !valid_offsets(src_off, n_pairs) || !valid_offsets(tgt_off, n_pairs))
        return 0;
    Carver c(nullptr, ~(size_t)0 >> 1);
    IcpStore s;
    carve_batched(c, n_pairs, src_off, tgt_off, max_iters_max, s, nullptr, nullptr);
    return c.used();
}

namespace {

// batched point-to-plane ICP in a workspace region (arguments already checked)
pc_status batched_core(int n_pairs, const float *src_xyz, const int64_t *src_off, const float *tgt_xyz,
                       const float *tgt_normals, const int64_t *tgt_off, const double *init_T,
                       const float *max_corr_dist, const int32_t *max_iters, int iters_max, double conv_tol,
                       double *out_T, pc_icp_stats *out_stats, void *workspace, size_t workspace_bytes,
                       hipStream_t stream)
{
    Carver c(workspace, workspace_bytes);
    IcpStore s;
    std::vector<int32_t> boff, goff;
    carve_batched(c, n_pairs, src_off, tgt_off, iters_max, s, &boff, &goff);
    if (!c.ok) return PC_EWORKSPACE;
    if (!upload(s.soff, src_off, sizeof(int64_t) * (n_pairs + 1), stream) ||
        !upload(s.grid.off, tgt_off, sizeof(int64_t) * (n_pairs + 1), stream) ||
        !upload(s.boff, boff.data(), sizeof(int32_t) * (n_pairs + 1), stream) ||
        !upload(s.goff, goff.data(), sizeof(int32_t) * (n_pairs + 1), stream) ||
        !upload(s.dmax, max_corr_dist, sizeof(float) * n_pairs, stream) ||
        !upload(s.maxit, max_iters, sizeof(int32_t) * n_pairs, stream))
        return PC_EDEVICE;
    hipError_t e = icp_run(s, src_xyz, src_off[n_pairs], tgt_xyz, tgt_normals, init_T, conv_tol, out_T, out_stats,
                           stream);
    return e == hipSuccess ? PC_OK : PC_EDEVICE;
}

}  // namespace

pc_status icp_point_to_plane_batched(int n_pairs, const float *src_xyz, const int64_t *src_off,
                                     const float *tgt_xyz, const float *tgt_normals, const int64_t *tgt_off,
                                     const double *init_T, const float *max_corr_dist, const int32_t *max_iters,
                                     double conv_tol, double *out_T, pc_icp_stats *out_stats, void *workspace,
                                     size_t workspace_bytes, hipStream_t stream)
{
    if (n_pairs < 1 || !valid_offsets(src_off, n_pairs) || !valid_offsets(tgt_off, n_pairs)) return PC_EINVAL;
    if (!max_corr_dist || !max_iters) return PC_EINVAL;
    int iters_max = 0;
    for (int p = 0; p < n_pairs; p++) {
        if (max_iters[p] < 0 || !(max_corr_dist[p] > 0.f) || !isfinite(max_corr_dist[p])) return PC_EINVAL;
        iters_max = max_iters[p] > iters_max ? max_iters[p] : iters_max;
    }
    if (!(conv_tol >= 0.0) || !isfinite(conv_tol)) return PC_EINVAL;
    const int64_t ns = src_off[n_pairs], nt = tgt_off[n_pairs];
    if (!out_T || !workspace) return PC_EINVAL;
    if ((ns > 0 && !src_xyz) || (nt > 0 && (!tgt_xyz || !tgt_normals))) return PC_EINVAL;
    if (!aligned(src_xyz, 4) || !aligned(tgt_xyz, 4) || !aligned(tgt_normals, 4) || !aligned(init_T, 8) ||
        !aligned(out_T, 8) || !aligned(out_stats, 8) || !aligned(workspace, 256))
        return PC_EINVAL;
    if (workspace_bytes < icp_point_to_plane_batched_workspace_size(n_pairs, src_off, tgt_off, iters_max))
        return PC_EWORKSPACE;
    return batched_core(n_pairs, src_xyz, src_off, tgt_xyz, tgt_normals, tgt_off, init_T, max_corr_dist, max_iters,
                        iters_max, conv_tol, out_T, out_stats, workspace, workspace_bytes, stream);
}

size_t icp_point_to_plane_with_normals_batched_workspace_size(int n_pairs, const int64_t *src_off,
                                                              const int64_t *tgt_off, int max_iters_max)
{
    if (n_pairs < 1 || max_iters_max < 0 || !valid_offsets(src_off, n_pairs) || !valid_offsets(tgt_off, n_pairs))
        return 0;
    Carver c(nullptr, ~(size_t)0 >> 1);
    IcpStore s;
    carve_batched(c, n_pairs, src_off, tgt_off, max_iters_max, s, nullptr, nullptr);
    c.take<float>((size_t)3 * (tgt_off[n_pairs] > 0 ? tgt_off[n_pairs] : 1));
    c.take<int32_t>((size_t)n_pairs);
    return c.used();
}

pc_status icp_point_to_plane_with_normals_batched(int n_pairs, const float *src_xyz, const int64_t *src_off,
                                                  const float *tgt_xyz, const int64_t *tgt_off, const int32_t *k,
                                                  const float viewpoint[3], const double *init_T,
                                                  const float *max_corr_dist, const int32_t *max_iters,
                                                  double conv_tol, double *out_T, pc_icp_stats *out_stats,
                                                  float *out_normals, void *workspace, size_t workspace_bytes,
                                                  hipStream_t stream)
{
    if (n_pairs < 1 || !valid_offsets(src_off, n_pairs) || !valid_offsets(tgt_off, n_pairs)) return PC_EINVAL;
    if (!max_corr_dist || !max_iters || !k || !viewpoint) return PC_EINVAL;
    int iters_max = 0, k_max = 1;
    for (int p = 0; p < n_pairs; p++) {
        if (max_iters[p] < 0 || !(max_corr_dist[p] > 0.f) || !isfinite(max_corr_dist[p])) return PC_EINVAL;
        iters_max = max_iters[p] > iters_max ? max_iters[p] : iters_max;
        const int64_t nc = tgt_off[p + 1] - tgt_off[p];
        if (k[p] < 1 || k[p] > PCGPU_KMAX || (nc > 0 && k[p] > nc)) return PC_EINVAL;
        k_max = k[p] > k_max ? k[p] : k_max;
    }
    if (!isfinite(viewpoint[0]) || !isfinite(viewpoint[1]) || !isfinite(viewpoint[2])) return PC_EINVAL;
    if (!(conv_tol >= 0.0) || !isfinite(conv_tol)) return PC_EINVAL;
    const int64_t ns = src_off[n_pairs], nt = tgt_off[n_pairs];
    if (!out_T || !workspace) return PC_EINVAL;
    if ((ns > 0 && !src_xyz) || (nt > 0 && !tgt_xyz)) return PC_EINVAL;
    if (!aligned(src_xyz, 4) || !aligned(tgt_xyz, 4) || !aligned(out_normals, 4) || !aligned(init_T, 8) ||
        !aligned(out_T, 8) || !aligned(out_stats, 8) || !aligned(workspace, 256))
        return PC_EINVAL;
    if (workspace_bytes < icp_point_to_plane_with_normals_batched_workspace_size(n_pairs, src_off, tgt_off, iters_max))
        return PC_EWORKSPACE;
    Carver c(workspace, workspace_bytes);
    IcpStore s;
    std::vector<int32_t> boff, goff;
    carve_batched(c, n_pairs, src_off, tgt_off, iters_max, s, &boff, &goff);
    float *nb = c.take<float>((size_t)3 * (nt > 0 ? nt : 1));
    int32_t *kc = c.take<int32_t>((size_t)n_pairs);
    if (!c.ok) return PC_EWORKSPACE;
    if (out_normals) nb = out_normals;
    if (!upload(s.soff, src_off, sizeof(int64_t) * (n_pairs + 1), stream) ||
        !upload(s.grid.off, tgt_off, sizeof(int64_t) * (n_pairs + 1), stream) ||
        !upload(s.boff, boff.data(), sizeof(int32_t) * (n_pairs + 1), stream) ||
        !upload(s.goff, goff.data(), sizeof(int32_t) * (n_pairs + 1), stream) ||
        !upload(s.dmax, max_corr_dist, sizeof(float) * n_pairs, stream) ||
        !upload(s.maxit, max_iters, sizeof(int32_t) * n_pairs, stream) ||
        !upload(kc, k, sizeof(int32_t) * n_pairs, stream))
        return PC_EDEVICE;
    // one pyramid over the targets serves their normals and the correspondences
    if (grid_build(s.grid, tgt_xyz, stream) != hipSuccess) return PC_EDEVICE;
    if (nt > 0 &&
        normals_run(s.grid, tgt_xyz, k_max, kc, viewpoint, nb, nullptr, stream, INFINITY, 0, s.nrm) != hipSuccess)
        return PC_EDEVICE;
    s.grid_built = true;
    s.nrm_ready = true;
    hipError_t e = icp_run(s, src_xyz, ns, tgt_xyz, nb, init_T, conv_tol, out_T, out_stats, stream);
    return e == hipSuccess ? PC_OK : PC_EDEVICE;
}

// ---------------------------------------------------------------------------
// Learned pose initialiser and multi-start ICP
// ---------------------------------------------------------------------------
namespace {

// per cloud row ranges (source p -> cloud 2p, target p -> cloud 2p + 1) and
// encoder tile offsets
bool pose_layout(int n_pairs, const int64_t *src_off, const int64_t *tgt_off, std::vector<int64_t> &cr,
                 std::vector<int32_t> &toff, int &ntile)
{
    cr.assign((size_t)4 * n_pairs, 0);
    toff.assign((size_t)2 * n_pairs + 1, 0);
    int64_t tiles = 0;
    for (int p = 0; p < n_pairs; p++) {
        cr[4 * p] = src_off[p];
        cr[4 * p + 1] = src_off[p + 1];
        cr[4 * p + 2] = tgt_off[p];
        cr[4 * p + 3] = tgt_off[p + 1];
        tiles += pose_net_tiles(src_off[p + 1] - src_off[p]);
        toff[2 * p + 1] = (int32_t)tiles;
        tiles += pose_net_tiles(tgt_off[p + 1] - tgt_off[p]);
        toff[2 * p + 2] = (int32_t)tiles;
        if (tiles >= ((int64_t)1 << 30)) return false;
    }
    ntile = (int)tiles;
    return true;
}

bool pose_args_ok(int n_pairs, const float *src_xyz, const int64_t *src_off, const float *tgt_xyz,
                  const int64_t *tgt_off)
{
    // the encoder alone has no search structure, so no cloud limit of its own
    if (n_pairs < 1 || n_pairs > (1 << 24) || !valid_offsets(src_off, n_pairs, 1 << 24) ||
        !valid_offsets(tgt_off, n_pairs, 1 << 24))
        return false;
    if ((src_off[n_pairs] > 0 && !src_xyz) || (tgt_off[n_pairs] > 0 && !tgt_xyz)) return false;
    return aligned(src_xyz, 4) && aligned(tgt_xyz, 4);
}

size_t pose_store_bytes(int n_pairs, int ntile, bool train)
{
    Carver c(nullptr, ~(size_t)0 >> 1);
    PoseNetStore s;
    pose_net_carve(c, n_pairs, ntile, train, s);
    return c.used();
}

// the pairs' offsets to the device (half the bytes of the per-cloud rows
// and tile offsets, so fewer upload launches), expanded there into both
pc_status pose_upload_layout(int n_pairs, const int64_t *src_off, const int64_t *tgt_off, PoseNetStore &s,
                             hipStream_t stream)
{
    std::vector<int64_t> offs(src_off, src_off + n_pairs + 1);
    offs.insert(offs.end(), tgt_off, tgt_off + n_pairs + 1);
    if (!upload(s.offs, offs.data(), sizeof(int64_t) * offs.size(), stream)) return PC_EDEVICE;
    return pose_net_layout(s, stream) == hipSuccess ? PC_OK : PC_EDEVICE;
}

// carve the pose store at the front of the workspace and upload its layout
pc_status pose_setup(Carver &c, int n_pairs, const int64_t *src_off, const int64_t *tgt_off, bool train,
                     PoseNetStore &s, hipStream_t stream)
{
    std::vector<int64_t> cr;
    std::vector<int32_t> toff;
    int ntile = 0;
    if (!pose_layout(n_pairs, src_off, tgt_off, cr, toff, ntile)) return PC_EINVAL;
    pose_net_carve(c, n_pairs, ntile, train, s);
    if (!c.ok) return PC_EWORKSPACE;
    return pose_upload_layout(n_pairs, src_off, tgt_off, s, stream);
}

// replicated offsets of every pair kStarts times (pair-major)
void replicate_offsets(int n, const int32_t *sel, const int64_t *off, std::vector<int64_t> &rep)
{
    rep.assign(1, 0);
    for (int i = 0; i < n; i++) {
        const int p = sel ? sel[i] : i;
        for (int j = 0; j < kStarts; j++) rep.push_back(rep.back() + (off[p + 1] - off[p]));
    }
}

struct LearnedLayout {
    PoseNetStore pose;
    pc_icp_stats *st1, *st_all;
    int32_t *sel;
    int64_t *seg_s, *seg_t;
    float *rs, *rt, *rn;
    double *T_start, *T_all;
    void *icp;
    size_t icp_bytes;
};

size_t icp_region_bytes(int n_pairs, const int64_t *src_off, const int64_t *tgt_off, int max_iters)
{
    std::vector<int64_t> rs, rt;
    replicate_offsets(n_pairs, nullptr, src_off, rs);
    replicate_offsets(n_pairs, nullptr, tgt_off, rt);
    size_t a = icp_point_to_plane_batched_workspace_size(n_pairs, src_off, tgt_off, max_iters);
    size_t b = icp_point_to_plane_batched_workspace_size(kStarts * n_pairs, rs.data(), rt.data(), max_iters);
    return a > b ? a : b;
}

// everything but the pose store's layout upload; returns false when the
// workspace is too small
bool learned_carve(Carver &c, int n_pairs, const int64_t *src_off, const int64_t *tgt_off, int max_iters, int ntile,
                   LearnedLayout &L)
{
    pose_net_carve(c, n_pairs, ntile, false, L.pose);
    const int64_t ns = src_off[n_pairs], nt = tgt_off[n_pairs];
    const size_t R = (size_t)kStarts * n_pairs;
    L.st1 = c.take<pc_icp_stats>(n_pairs);
    L.st_all = c.take<pc_icp_stats>(R);
    L.sel = c.take<int32_t>(n_pairs);
    L.seg_s = c.take<int64_t>(3 * R);
    L.seg_t = c.take<int64_t>(3 * R);
    L.rs = c.take<float>((size_t)3 * kStarts * ns);
    L.rt = c.take<float>((size_t)3 * kStarts * nt);
    L.rn = c.take<float>((size_t)3 * kStarts * nt);
    L.T_start = c.take<double>(16 * R);
    L.T_all = c.take<double>(16 * R);
    L.icp_bytes = icp_region_bytes(n_pairs, src_off, tgt_off, max_iters);
    L.icp = c.take<uint8_t>(L.icp_bytes);
    return c.ok;
}

}  // namespace

int pose_net_param_count(void) { return kParams; }

size_t pose_net_workspace_size(int n_pairs, const int64_t *src_off, const int64_t *tgt_off)
{
    std::vector<int64_t> cr;
    std::vector<int32_t> toff;
    int ntile = 0;
    if (n_pairs < 1 || n_pairs > (1 << 24) || !valid_offsets(src_off, n_pairs, 1 << 24) ||
        !valid_offsets(tgt_off, n_pairs, 1 << 24))
        return 0;
    if (!pose_layout(n_pairs, src_off, tgt_off, cr, toff, ntile)) return 0;
    return pose_store_bytes(n_pairs, ntile, true);
}

pc_status pose_net_predict(const float *params, int n_pairs, const float *src_xyz, const int64_t *src_off,
                           const float *tgt_xyz, const int64_t *tgt_off, double *out_T, void *workspace,
                           size_t workspace_bytes, hipStream_t stream)
{
    if (!params || !aligned(params, 4) || !pose_args_ok(n_pairs, src_xyz, src_off, tgt_xyz, tgt_off)) return PC_EINVAL;
    if (!out_T || !aligned(out_T, 8) || !workspace || !aligned(workspace, 256)) return PC_EINVAL;
    if (workspace_bytes < pose_net_workspace_size(n_pairs, src_off, tgt_off)) return PC_EWORKSPACE;
    Carver c(workspace, workspace_bytes);
    PoseNetStore s;
    pc_status r = pose_setup(c, n_pairs, src_off, tgt_off, false, s, stream);
    if (r != PC_OK) return r;
    // kernel timer slot 0: the encoder kernel
    return pose_net_forward(s, params, src_xyz, tgt_xyz, out_T, stream, 0) == hipSuccess ? PC_OK : PC_EDEVICE;
}

pc_status pose_net_train_step(float *params, float *adam_m, float *adam_v, int step, float lr, int n_pairs,
                              const float *src_xyz, const int64_t *src_off, const float *tgt_xyz,
                              const int64_t *tgt_off, const double *label_T, const float *pair_weight,
                              float *out_loss, float *out_grad, void *workspace, size_t workspace_bytes,
                              hipStream_t stream)
{
    if (!params || !aligned(params, 4) || !pose_args_ok(n_pairs, src_xyz, src_off, tgt_xyz, tgt_off)) return PC_EINVAL;
    if (step < 1 || !(lr >= 0.f) || !isfinite(lr)) return PC_EINVAL;
    if (lr > 0.f && (!adam_m || !adam_v || !aligned(adam_m, 4) || !aligned(adam_v, 4))) return PC_EINVAL;
    if (!label_T || !aligned(label_T, 8) || !aligned(pair_weight, 4) || !aligned(out_loss, 4) ||
        !aligned(out_grad, 4))
        return PC_EINVAL;
    if (!workspace || !aligned(workspace, 256)) return PC_EINVAL;
    if (workspace_bytes < pose_net_workspace_size(n_pairs, src_off, tgt_off)) return PC_EWORKSPACE;
    Carver c(workspace, workspace_bytes);
    PoseNetStore s;
    pc_status r = pose_setup(c, n_pairs, src_off, tgt_off, true, s, stream);
    if (r != PC_OK) return r;
    if (pose_net_train(s, params, adam_m, adam_v, step, lr, src_xyz, tgt_xyz, label_T, pair_weight, out_loss,
                       stream) != hipSuccess)
        return PC_EDEVICE;
    if (out_grad && hipMemcpyAsync(out_grad, s.grad, sizeof(float) * kParams, hipMemcpyDeviceToDevice, stream) !=
                        hipSuccess)
        return PC_EDEVICE;
    return PC_OK;
}

size_t icp_learned_batched_workspace_size(int n_pairs, const int64_t *src_off, const int64_t *tgt_off,
                                          int max_iters)
{
    std::vector<int64_t> cr;
    std::vector<int32_t> toff;
    int ntile = 0;
    if (n_pairs < 1 || max_iters < 0 || !valid_offsets(src_off, n_pairs) || !valid_offsets(tgt_off, n_pairs))
        return 0;
    if ((int64_t)kStarts * src_off[n_pairs] >= kMaxPoints || (int64_t)kStarts * tgt_off[n_pairs] >= kMaxPoints)
        return 0;
    if ((int64_t)kStarts * n_pairs > PCGPU_MAX_CLOUDS) return 0;   // the replicated multi-start batch
    if (!pose_layout(n_pairs, src_off, tgt_off, cr, toff, ntile)) return 0;
    Carver c(nullptr, ~(size_t)0 >> 1);
    LearnedLayout L;
    learned_carve(c, n_pairs, src_off, tgt_off, max_iters, ntile, L);
    return c.used();
}

pc_status icp_learned_batched(int mode, const float *params, int n_pairs, const float *src_xyz,
                              const int64_t *src_off, const float *tgt_xyz, const float *tgt_normals,
                              const int64_t *tgt_off, float max_corr_dist, int max_iters, double conv_tol,
                              float accept_rms, double *out_T, pc_icp_stats *out_stats, int32_t *out_start,
                              void *workspace, size_t workspace_bytes, hipStream_t stream)
{
    if (mode != PC_INIT_LEARNED && mode != PC_INIT_MULTI_START && mode != PC_INIT_LEARNED_ONLY) return PC_EINVAL;
    if (mode != PC_INIT_MULTI_START && (!params || !aligned(params, 4))) return PC_EINVAL;
    if (!pose_args_ok(n_pairs, src_xyz, src_off, tgt_xyz, tgt_off)) return PC_EINVAL;
    if (tgt_off[n_pairs] > 0 && (!tgt_normals || !aligned(tgt_normals, 4))) return PC_EINVAL;
    if (max_iters < 0 || !(max_corr_dist > 0.f) || !isfinite(max_corr_dist)) return PC_EINVAL;
    if (!(conv_tol >= 0.0) || !isfinite(conv_tol) || isnan(accept_rms)) return PC_EINVAL;
    if (!out_T || !aligned(out_T, 8) || !aligned(out_stats, 8) || !aligned(out_start, 4)) return PC_EINVAL;
    if (!workspace || !aligned(workspace, 256)) return PC_EINVAL;
    const size_t need = icp_learned_batched_workspace_size(n_pairs, src_off, tgt_off, max_iters);
    if (need == 0) return PC_EINVAL;
    if (workspace_bytes < need) return PC_EWORKSPACE;

    Carver c(workspace, workspace_bytes);
    LearnedLayout L;
    std::vector<int64_t> cr;
    std::vector<int32_t> toff;
    int ntile = 0;
    if (!pose_layout(n_pairs, src_off, tgt_off, cr, toff, ntile)) return PC_EINVAL;
    if (!learned_carve(c, n_pairs, src_off, tgt_off, max_iters, ntile, L)) return PC_EWORKSPACE;
    if (pose_upload_layout(n_pairs, src_off, tgt_off, L.pose, stream) != PC_OK) return PC_EDEVICE;
    std::vector<float> dmax(kStarts * (size_t)n_pairs, max_corr_dist);
    std::vector<int32_t> maxit(kStarts * (size_t)n_pairs, max_iters);
    if (out_start && fill_i32(out_start, n_pairs, -1, stream) != hipSuccess) return PC_EDEVICE;

    std::vector<int32_t> sel;
    if (mode == PC_INIT_MULTI_START) {
        if (pose_net_stats(L.pose, src_xyz, tgt_xyz, stream) != hipSuccess) return PC_EDEVICE;
        for (int p = 0; p < n_pairs; p++) sel.push_back(p);
    } else {
        // learned initial pose, then ICP from it
        if (pose_net_forward(L.pose, params, src_xyz, tgt_xyz, L.pose.T, stream) != hipSuccess) return PC_EDEVICE;
        pc_status r = batched_core(n_pairs, src_xyz, src_off, tgt_xyz, tgt_normals, tgt_off, L.pose.T, dmax.data(),
                                   maxit.data(), max_iters, conv_tol, out_T, L.st1, L.icp, L.icp_bytes, stream);
        if (r != PC_OK) return r;
        if (out_stats && hipMemcpyAsync(out_stats, L.st1, sizeof(pc_icp_stats) * n_pairs, hipMemcpyDeviceToDevice,
                                        stream) != hipSuccess)
            return PC_EDEVICE;
        if (mode == PC_INIT_LEARNED_ONLY) return PC_OK;
        // pairs whose refinement did not reach the accepted residual
        std::vector<pc_icp_stats> h(n_pairs);
        if (hipMemcpyAsync(h.data(), L.st1, sizeof(pc_icp_stats) * n_pairs, hipMemcpyDeviceToHost, stream) !=
                hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
            return PC_EDEVICE;
        for (int p = 0; p < n_pairs; p++) {
            const pc_icp_stats &t = h[p];
            const bool ok = (t.status == PC_ICP_CONVERGED || t.status == PC_ICP_MAXITER) && t.inliers > 0 &&
                            t.rms <= (double)accept_rms;
            if (!ok) sel.push_back(p);
        }
    }
    const int F = (int)sel.size();
    if (F == 0) return PC_OK;
    // the selected pairs, each kStarts times, gathered into contiguous clouds
    std::vector<int64_t> rso, rto, seg_s, seg_t;
    replicate_offsets(F, sel.data(), src_off, rso);
    replicate_offsets(F, sel.data(), tgt_off, rto);
    for (int i = 0; i < F; i++)
        for (int j = 0; j < kStarts; j++) {
            const int p = sel[i], r = i * kStarts + j;
            seg_s.insert(seg_s.end(), {rso[r], src_off[p], src_off[p + 1] - src_off[p]});
            seg_t.insert(seg_t.end(), {rto[r], tgt_off[p], tgt_off[p + 1] - tgt_off[p]});
        }
    const int R = F * kStarts;
    if (!upload(L.sel, sel.data(), sizeof(int32_t) * F, stream) ||
        !upload(L.seg_s, seg_s.data(), sizeof(int64_t) * seg_s.size(), stream) ||
        !upload(L.seg_t, seg_t.data(), sizeof(int64_t) * seg_t.size(), stream))
        return PC_EDEVICE;
    if (gather_rows3(src_xyz, L.rs, L.seg_s, R, stream) != hipSuccess ||
        gather_rows3(tgt_xyz, L.rt, L.seg_t, R, stream) != hipSuccess ||
        gather_rows3(tgt_normals, L.rn, L.seg_t, R, stream) != hipSuccess ||
        multi_start_poses(L.pose.cen, L.sel, F, L.T_start, stream) != hipSuccess)
        return PC_EDEVICE;
    pc_status r = batched_core(R, L.rs, rso.data(), L.rt, L.rn, rto.data(), L.T_start, dmax.data(), maxit.data(),
                               max_iters, conv_tol, L.T_all, L.st_all, L.icp, L.icp_bytes, stream);
    if (r != PC_OK) return r;
    return multi_start_select(L.T_all, L.st_all, L.sel, F, out_T, out_stats, out_start, stream) == hipSuccess
               ? PC_OK
               : PC_EDEVICE;
}

const double *icp_history(void *workspace, size_t workspace_bytes, int64_t n_src, int64_t n_tgt, int max_iters)
{
    if (!workspace || workspace_bytes < icp_point_to_plane_workspace_size(n_src, n_tgt, max_iters)) return nullptr;
    Carver c(workspace, workspace_bytes);
    IcpStore s;
    carve_single(c, n_src, n_tgt, max_iters, s);
    return s.hist;
}

pc_status pc_copy_probe(void *dst, const void *src, size_t n_bytes, hipStream_t stream)
{
    if (!dst || !src || n_bytes % 16 || !aligned(dst, 16) || !aligned(src, 16)) return PC_EINVAL;
    size_t n = n_bytes / 16;
    if (n == 0) return PC_OK;
    int blocks = (int)((n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192);
    k_copy16<<<blocks, 256, 0, stream>>>((const uint4 *)src, (uint4 *)dst, n);
    return hipGetLastError() == hipSuccess ? PC_OK : PC_EDEVICE;
}

pc_status pc_set_kernel_timer(hipEvent_t *begin, hipEvent_t *end, int capacity)
{
    if (capacity < 0 || (capacity > 0 && (!begin || !end))) return PC_EINVAL;
    icp_set_timer(begin, end, capacity);
    return PC_OK;
}

int pc_kernel_timer_count(void) { return icp_timer_count(); }

pc_status pc_set_tuning(const pc_tuning *t)
{
    if (!t) return PC_EINVAL;
    int b = t->icp_block_threads, l = t->icp_leaf;
    if (b != 64 && b != 128 && b != 256) return PC_EINVAL;
    if (l != 8 && l != 16 && l != 32) return PC_EINVAL;
    if (!(t->node_budget >= 0.125f && t->node_budget <= 1.0f)) return PC_EINVAL;
    if (t->sort_queries != 0 && t->sort_queries != 1) return PC_EINVAL;
    // The persistent form of the ICP loop (k_icp_persistent) is switched
    // off: after the search's register allocation changed, a run of it
    // stopped making progress, and the cause is not established.  The
    // knob accepts 0 only; the kernel stays in the source, unreachable.
    if (t->icp_persistent != 0) return PC_EINVAL;
    g_tune = *t;
    return PC_OK;
}

void pc_get_tuning(pc_tuning *t)
{
    if (t) *t = g_tune;
}

}  // extern "C"
