// C-ABI entry points: argument validation, workspace carving, launches.

#include <math.h>

#include <vector>

#include "icp.h"

using namespace pcg;

namespace {

constexpr int64_t kMaxPoints = (int64_t)1 << 31;

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

// host offsets of m items: off[0] = 0, non-decreasing, total below kMaxPoints
bool valid_offsets(const int64_t *off, int m)
{
    if (!off || m < 1 || off[0] != 0) return false;
    for (int i = 0; i < m; i++)
        if (off[i + 1] < off[i]) return false;
    return off[m] < kMaxPoints;
}

// process-wide tuning of the ICP kernels and the pyramid (pc_set_tuning)
pc_tuning g_tune = {128, 16, 1.0f};

bool upload(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    return bytes == 0 || hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s) == hipSuccess;
}

__global__ void k_copy16(const uint4 *__restrict__ src, uint4 *__restrict__ dst, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
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
}

// the single-pair carve, shared by the size query, the call and the history
void carve_single(Carver &c, int64_t n_src, int64_t n_tgt, int max_iters, IcpStore &s)
{
    int64_t cap = icp_blocks_max(n_src);
    icp_carve(c, 1, n_src, n_tgt, cap, icp_groups(cap), max_iters, s);
    tune(s);
    s.nblk = (int)icp_blocks(n_src, s.threads);
    s.ngrp = (int)icp_groups(s.nblk);
}

// the batched carve: blocks and groups per pair from the host offsets
void carve_batched(Carver &c, int n_pairs, const int64_t *src_off, const int64_t *tgt_off, int iters_max,
                   IcpStore &s, std::vector<int32_t> *boff, std::vector<int32_t> *goff)
{
    int64_t cap_b = 0, cap_g = 0, nblk = 0, ngrp = 0;
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
        if (boff) boff->push_back((int32_t)nblk);
        if (goff) goff->push_back((int32_t)ngrp);
    }
    icp_carve(c, n_pairs, src_off[n_pairs], tgt_off[n_pairs], cap_b, cap_g, iters_max, s);
    tune(s);
    s.nblk = (int)nblk;
    s.ngrp = (int)ngrp;
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

// single-pair ICP with any metric (0 point-to-plane, 1 point-to-point, 2 combined)
pc_status icp_single(const float *src_xyz, int64_t n_src, const float *tgt_xyz, const float *tgt_normals,
                     int64_t n_tgt, const double *init_T, float max_corr_dist, int max_iters, double conv_tol,
                     double *out_T, pc_icp_stats *out_stats, void *workspace, size_t workspace_bytes,
                     hipStream_t stream, int metric, float w_point, float w_plane)
{
    const bool need_normals = metric == 0 || (metric == 2 && w_plane > 0.f);
    if (n_src < 0 || n_tgt < 0 || n_src >= kMaxPoints || n_tgt >= kMaxPoints) return PC_EINVAL;
    if (max_iters < 0 || !(max_corr_dist > 0.f) || !isfinite(max_corr_dist)) return PC_EINVAL;
    if (!(conv_tol >= 0.0) || !isfinite(conv_tol)) return PC_EINVAL;
    if (!out_T || !workspace) return PC_EINVAL;
    if ((n_src > 0 && !src_xyz) || (n_tgt > 0 && (!tgt_xyz || (need_normals && !tgt_normals)))) return PC_EINVAL;
    if (!aligned(src_xyz, 4) || !aligned(tgt_xyz, 4) || !aligned(tgt_normals, 4) || !aligned(init_T, 8) ||
        !aligned(out_T, 8) || !aligned(out_stats, 8) || !aligned(workspace, 256))
        return PC_EINVAL;
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
    hipError_t e = icp_run(s, src_xyz, ns, tgt_xyz, tgt_normals, init_T, conv_tol, out_T, out_stats, stream);
    return e == hipSuccess ? PC_OK : PC_EDEVICE;
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
    g_tune = *t;
    return PC_OK;
}

void pc_get_tuning(pc_tuning *t)
{
    if (t) *t = g_tune;
}

}  // extern "C"
