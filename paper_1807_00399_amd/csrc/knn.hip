// k-nearest-neighbour queries and PCA normals on the sparse voxel pyramid.
//
// k-NN (Section 3, "Core operations"): exact k nearest reference points of
// each query under the float32 key, ties to the lower original index.
// Normals (Section 3, "Core operations": normal and curvature estimation via
// PCA; Section 4: 10-NN neighbourhoods, viewpoint-consistent orientation):
// the k-NN of every point in its own cloud, their covariance, the unit
// eigenvector of its smallest eigenvalue flipped toward the viewpoint, and
// the surface variation l0/(l0+l1+l2).  The neighbour search and all loads
// run in float32; the covariance is accumulated in float64 from the exact
// query-relative offsets and decomposed with the closed-form trigonometric
// eigenvalues of a symmetric 3x3 matrix (Smith 1961) and a cross product of
// two rows of (C - l0 I) for the eigenvector (Kopp 2008).  The eigenvector
// error of any solver scales as eps * l2 / (l1 - l0); float64 keeps it far
// below 1e-5 rad wherever the normal is well defined.

#include "icp.h"
#include "search.h"

namespace pcg {

namespace {

// one wave per block: the blocks of uneven search lengths retire and refill
// independently (street and batch normals ~8 % faster than 256 threads)
constexpr int kQThreads = 64;

template <int KT, int LEAF>
__global__ void __launch_bounds__(kQThreads) k_knn(GridView g, const float *__restrict__ qry, int64_t nq, int k,
                                                 int32_t *__restrict__ out_idx, float *__restrict__ out_d2)
{
    __shared__ __align__(8) uint32_t stk[SearchStack::words * kQThreads];
    const GridParams P = g.params[0];   // the reference cloud
    int64_t i = xcd_block(blockIdx.x, gridDim.x) * (int64_t)kQThreads + threadIdx.x;
    if (i >= nq) return;
    Query q{qry[3 * i], qry[3 * i + 1], qry[3 * i + 2]};
    const int32_t seed = search_seed(g, P, q, k, INFINITY);   // before the list is set up
    TopK<KT> top;
    top.init(k);
    search_from<TopK<KT>, LEAF>(g, P, q, top, seed, lane_stack<SearchStack>(stk, kQThreads));
#pragma unroll
    for (int s = 0; s < KT; s++) {
        if (s >= KT - k) {
            int o = s - (KT - k);
            out_idx[i * k + o] = (int32_t)(uint32_t)top.h[s];
            if (out_d2) out_d2[i * k + o] = __uint_as_float((uint32_t)(top.h[s] >> 32));
        }
    }
}

// eigen-decomposition of the symmetric C = [a b c; b d e; c e f] (float64):
// ascending eigenvalues and the unit eigenvector of the smallest.  Written
// with selects only, so everything stays in registers.
__device__ void sym3_min_eigvec(double a, double b, double c, double d, double e, double f, double lam[3],
                                double v[3])
{
    double p1 = b * b + c * c + e * e;
    if (p1 == 0.0) {
        // diagonal: smallest entry, lowest axis first on ties
        int i0 = (d < a) ? 1 : 0;
        double m0 = (d < a) ? d : a;
        i0 = (f < m0) ? 2 : i0;
        double lo = (f < m0) ? f : m0;
        double hi = fmax(a, fmax(d, f));
        lam[0] = lo;
        lam[2] = hi;
        lam[1] = (a + d + f) - lo - hi;
        v[0] = i0 == 0 ? 1.0 : 0.0;
        v[1] = i0 == 1 ? 1.0 : 0.0;
        v[2] = i0 == 2 ? 1.0 : 0.0;
        return;
    }
    double q = (a + d + f) / 3.0;
    double ba = a - q, bd = d - q, bf = f - q;
    double p2 = ba * ba + bd * bd + bf * bf + 2.0 * p1;
    double p = sqrt(p2 / 6.0);
    double det = ba * (bd * bf - e * e) - b * (b * bf - e * c) + c * (b * e - bd * c);
    double r = det / (2.0 * p * p * p);
    r = r < -1.0 ? -1.0 : (r > 1.0 ? 1.0 : r);
    double phi = acos(r) / 3.0;
    double l2 = q + 2.0 * p * cos(phi);
    double l0 = q + 2.0 * p * cos(phi + 2.0943951023931954923);   // + 2 pi / 3
    double l1 = 3.0 * q - l0 - l2;
    lam[0] = l0;
    lam[1] = l1;
    lam[2] = l2;
    // rows of C - l0 I and their pairwise cross products
    double r0x = a - l0, r0y = b, r0z = c;
    double r1x = b, r1y = d - l0, r1z = e;
    double r2x = c, r2y = e, r2z = f - l0;
    double ax = r0y * r1z - r0z * r1y, ay = r0z * r1x - r0x * r1z, az = r0x * r1y - r0y * r1x;
    double bx = r0y * r2z - r0z * r2y, by = r0z * r2x - r0x * r2z, bz = r0x * r2y - r0y * r2x;
    double cx = r1y * r2z - r1z * r2y, cy = r1z * r2x - r1x * r2z, cz = r1x * r2y - r1y * r2x;
    double na = ax * ax + ay * ay + az * az, nb = bx * bx + by * by + bz * bz, nc = cx * cx + cy * cy + cz * cz;
    double wx = ax, wy = ay, wz = az, nw = na;
    if (nb > nw) { wx = bx; wy = by; wz = bz; nw = nb; }
    if (nc > nw) { wx = cx; wy = cy; wz = cz; nw = nc; }
    double scale = fabs(l2) + fabs(l0);
    if (nw > 1e-60 * scale * scale * scale * scale && nw > 0.0) {
        double s = 1.0 / sqrt(nw);
        v[0] = wx * s;
        v[1] = wy * s;
        v[2] = wz * s;
        return;
    }
    // l0 (nearly) repeated: any unit vector orthogonal to the largest row of
    // (C - l0 I) lies in its eigenspace
    double gx = r0x, gy = r0y, gz = r0z, rn = r0x * r0x + r0y * r0y + r0z * r0z;
    double t1 = r1x * r1x + r1y * r1y + r1z * r1z, t2 = r2x * r2x + r2y * r2y + r2z * r2z;
    if (t1 > rn) { gx = r1x; gy = r1y; gz = r1z; rn = t1; }
    if (t2 > rn) { gx = r2x; gy = r2y; gz = r2z; rn = t2; }
    if (!(rn > 0.0)) {
        v[0] = 1.0; v[1] = 0.0; v[2] = 0.0;
        return;
    }
    // cross with the axis of the smallest component of that row
    int ax_i = 0;
    if (fabs(gy) < fabs(gx)) ax_i = 1;
    if (fabs(gz) < (ax_i == 0 ? fabs(gx) : fabs(gy))) ax_i = 2;
    double ex = ax_i == 0 ? 1.0 : 0.0, ey = ax_i == 1 ? 1.0 : 0.0, ez = ax_i == 2 ? 1.0 : 0.0;
    double ux = gy * ez - gz * ey, uy = gz * ex - gx * ez, uz = gx * ey - gy * ex;
    double s = 1.0 / sqrt(ux * ux + uy * uy + uz * uz);
    v[0] = ux * s;
    v[1] = uy * s;
    v[2] = uz * s;
}

// Normal and curvature of the point (qx, qy, qz) (original index qi) from
// its neighbourhood covariance: the unit eigenvector of the smallest
// eigenvalue, flipped toward the viewpoint (first nonzero component made
// positive when the product is exactly zero), curvature l0 / trace.  An
// all-zero covariance gives normal 0 and curvature 0.
__device__ void finish_normal(double cxx, double cxy, double cxz, double cyy, double cyz, double czz, double qx,
                              double qy, double qz, float vx, float vy, float vz, uint32_t qi,
                              float *__restrict__ out_n, float *__restrict__ out_c, float4 *srt_s = nullptr,
                              float gap = 0.f)
{
    double n[3] = {0.0, 0.0, 0.0}, lam[3] = {0.0, 0.0, 0.0};
    bool zero = cxx == 0.0 && cxy == 0.0 && cxz == 0.0 && cyy == 0.0 && cyz == 0.0 && czz == 0.0;
    if (!zero) {
        sym3_min_eigvec(cxx, cxy, cxz, cyy, cyz, czz, lam, n);
        double dot = n[0] * ((double)vx - qx) + n[1] * ((double)vy - qy) + n[2] * ((double)vz - qz);
        bool flip = dot < 0.0;
        if (dot == 0.0) {
            for (int a = 0; a < 3; a++)
                if (n[a] != 0.0) { flip = n[a] < 0.0; break; }
        }
        if (flip) { n[0] = -n[0]; n[1] = -n[1]; n[2] = -n[2]; }
    }
    out_n[3 * (int64_t)qi] = (float)n[0];
    out_n[3 * (int64_t)qi + 1] = (float)n[1];
    out_n[3 * (int64_t)qi + 2] = (float)n[2];
    if (srt_s) *srt_s = make_float4((float)n[0], (float)n[1], (float)n[2], gap);
    if (out_c) {
        double tr = lam[0] + lam[1] + lam[2];
        out_c[qi] = (float)(tr > 0.0 ? lam[0] / tr : 0.0);
    }
}

// One query per lane over every point of every cloud in the grid; the
// neighbourhood of a point is taken in its own cloud, with that cloud's k
// (kc[cloud], or k for all when kc is null).  With a finite cap2 (hybrid
// neighbourhoods) only neighbours with key <= cap2 count, and fewer than
// min_pts of them give normal 0.
// With srt, also the normal in sorted order with, in w, a lower bound of the
// squared distance to the nearest other point of the cloud (the second
// neighbour's key less 2^-20 relative; 0 when k < 2): the target record of
// the ICP correspondence search.
template <int KT, int LEAF>
__global__ void __launch_bounds__(kQThreads) k_normals(GridView g, int64_t n_all, const float *__restrict__ xyz, int k,
                                                     const int32_t *__restrict__ kc, float cap2, int min_pts,
                                                     float vx, float vy, float vz, float *__restrict__ out_n,
                                                     float *__restrict__ out_c, float4 *__restrict__ srt)
{
    __shared__ __align__(8) uint32_t stk[SearchStack::words * kQThreads];
    int64_t s = xcd_block(blockIdx.x, gridDim.x) * (int64_t)kQThreads + threadIdx.x;
    // queries are the points in sorted order, so neighbouring lanes search
    // neighbouring cells
    if (s >= n_all) return;
    const int cl = key_cloud(g.keys[s]);
    const GridParams P = g.params[cl];
    if (kc) k = kc[cl];
    float4 p = g.pts[s];
    uint32_t qi = __float_as_uint(p.w);
    Query q{p.x, p.y, p.z};
    const int32_t seed = search_seed(g, P, q, k, cap2);   // before the list is set up
    TopK<KT> top;
    top.init(k, cap2);
    search_from<TopK<KT>, LEAF>(g, P, q, top, seed, lane_stack<SearchStack>(stk, kQThreads));
    // the point itself (or an exact duplicate) is first, the nearest other
    // point second (selected with static indices: the list stays in registers)
    float gap = 0.f;
    if (srt) {
        uint64_t h2 = 0ull;
#pragma unroll
        for (int t = 1; t < KT; t++) h2 = (t == KT - k + 1) ? top.h[t] : h2;
        gap = h2 == ~0ull ? INFINITY : __uint_as_float((uint32_t)(h2 >> 32)) * (1.f - 1.f / (1 << 20));
    }
    // offsets from the query point are exact in float64 (differences of
    // float32 values); covariance is translation invariant.  One pass over
    // the neighbours (each one's coordinates gathered once): C = S / m -
    // mu mu^T from the sums of the offsets and of their products, whose
    // float64 cancellation error (~1e-16 of the neighbourhood's extent
    // squared) is far below the normal's tolerance.  Neighbours all at the
    // query give exactly zero.
    double qx = p.x, qy = p.y, qz = p.z;
    double sx = 0.0, sy = 0.0, sz = 0.0, sxx = 0.0, sxy = 0.0, sxz = 0.0, syy = 0.0, syz = 0.0, szz = 0.0;
    int m = 0;
#pragma unroll
    for (int t = 0; t < KT; t++) {
        if (t < KT - k) continue;
        uint32_t j = (uint32_t)top.h[t];
        if (j >= (uint32_t)n_all) continue;   // unfilled slot (only under a cap)
        m++;
        const double dx = (double)xyz[3 * (int64_t)j] - qx;
        const double dy = (double)xyz[3 * (int64_t)j + 1] - qy;
        const double dz = (double)xyz[3 * (int64_t)j + 2] - qz;
        sx += dx; sy += dy; sz += dz;
        sxx += dx * dx; sxy += dx * dy; sxz += dx * dz;
        syy += dy * dy; syz += dy * dz; szz += dz * dz;
    }
    if (m < min_pts || m == 0) {
        finish_normal(0.0, 0.0, 0.0, 0.0, 0.0, 0.0, qx, qy, qz, vx, vy, vz, qi, out_n, out_c, srt ? srt + s : nullptr, gap);
        return;
    }
    const double mx = sx / m, my = sy / m, mz = sz / m;
    double cxx = sxx / m - mx * mx, cxy = sxy / m - mx * my, cxz = sxz / m - mx * mz;
    double cyy = syy / m - my * my, cyz = syz / m - my * mz, czz = szz / m - mz * mz;
    finish_normal(cxx, cxy, cxz, cyy, cyz, czz, qx, qy, qz, vx, vy, vz, qi, out_n, out_c, srt ? srt + s : nullptr, gap);
}

// Radius neighbourhoods: every point of the cloud with key <= r2; the
// covariance from the one-pass sums, C = S / m - mu mu^T with mu = s / m;
// fewer than three points give normal 0.
template <int LEAF>
__global__ void __launch_bounds__(kQThreads) k_normals_radius(GridView g, int64_t n_all, float r2, float vx,
                                                            float vy, float vz, float *__restrict__ out_n,
                                                            float *__restrict__ out_c)
{
    __shared__ __align__(8) uint32_t stk[SearchStack::words * kQThreads];
    int64_t s = xcd_block(blockIdx.x, gridDim.x) * (int64_t)kQThreads + threadIdx.x;
    if (s >= n_all) return;
    const GridParams P = g.params[key_cloud(g.keys[s])];
    float4 p = g.pts[s];
    uint32_t qi = __float_as_uint(p.w);
    Query q{p.x, p.y, p.z};
    RadiusCov v;
    v.init(r2);
    search<RadiusCov, LEAF>(g, P, q, v, 1, lane_stack<SearchStack>(stk, kQThreads));
    double cxx = 0, cxy = 0, cxz = 0, cyy = 0, cyz = 0, czz = 0;
    if (v.m >= 3) {
        const double m = v.m, mx = v.sx / m, my = v.sy / m, mz = v.sz / m;
        cxx = v.sxx / m - mx * mx;
        cxy = v.sxy / m - mx * my;
        cxz = v.sxz / m - mx * mz;
        cyy = v.syy / m - my * my;
        cyz = v.syz / m - my * mz;
        czz = v.szz / m - mz * mz;
    }
    finish_normal(cxx, cxy, cxz, cyy, cyz, czz, p.x, p.y, p.z, vx, vy, vz, qi, out_n, out_c);
}

// Leaf size of the searches (nodes of at most LEAF points are scanned whole):
// smaller leaves visit more nodes and scan fewer points.  Results do not
// depend on it.
template <int KT, int LEAF>
void launch_knn_l(const GridStore &g, const float *qry, int64_t nq, int k, int32_t *oi, float *od, hipStream_t s)
{
    int blocks = (int)((nq + kQThreads - 1) / kQThreads);
    k_knn<KT, LEAF><<<blocks, kQThreads, 0, s>>>(g.view(), qry, nq, k, oi, od);
}

template <int KT>
void launch_knn(const GridStore &g, const float *qry, int64_t nq, int k, int32_t *oi, float *od, hipStream_t s)
{
    if (g.leaf <= 8) launch_knn_l<KT, 8>(g, qry, nq, k, oi, od, s);
    else if (g.leaf <= 16) launch_knn_l<KT, 16>(g, qry, nq, k, oi, od, s);
    else launch_knn_l<KT, 32>(g, qry, nq, k, oi, od, s);
}

template <int KT, int LEAF>
void launch_normals_l(const GridStore &g, const float *xyz, int k, const int32_t *kc, float cap2, int min_pts,
                      const float *vp, float *on, float *oc, float4 *srt, hipStream_t s)
{
    int blocks = (int)((g.n + kQThreads - 1) / kQThreads);
    k_normals<KT, LEAF><<<blocks, kQThreads, 0, s>>>(g.view(), g.n, xyz, k, kc, cap2, min_pts, vp[0], vp[1], vp[2],
                                                     on, oc, srt);
}

template <int KT>
void launch_normals(const GridStore &g, const float *xyz, int k, const int32_t *kc, float cap2, int min_pts,
                    const float *vp, float *on, float *oc, float4 *srt, hipStream_t s)
{
    if (g.leaf <= 8) launch_normals_l<KT, 8>(g, xyz, k, kc, cap2, min_pts, vp, on, oc, srt, s);
    else if (g.leaf <= 16) launch_normals_l<KT, 16>(g, xyz, k, kc, cap2, min_pts, vp, on, oc, srt, s);
    else launch_normals_l<KT, 32>(g, xyz, k, kc, cap2, min_pts, vp, on, oc, srt, s);
}

}  // namespace

hipError_t knn_run(const GridStore &g, const float *qry, int64_t nq, int k, int32_t *oi, float *od, hipStream_t s)
{
    if (nq <= 0) return hipSuccess;
    timer_search_begin(s);
    if (k <= 1) launch_knn<1>(g, qry, nq, k, oi, od, s);
    else if (k <= 4) launch_knn<4>(g, qry, nq, k, oi, od, s);
    else if (k <= 8) launch_knn<8>(g, qry, nq, k, oi, od, s);
    else if (k <= 16) launch_knn<16>(g, qry, nq, k, oi, od, s);
    else launch_knn<32>(g, qry, nq, k, oi, od, s);
    timer_search_end(s);
    return hipGetLastError();
}

hipError_t normals_run(const GridStore &g, const float *xyz, int k_max, const int32_t *kc, const float *vp,
                       float *on, float *oc, hipStream_t s, float cap2, int min_pts, float4 *srt)
{
    if (g.n <= 0) return hipSuccess;
    if (!(cap2 == INFINITY)) srt = nullptr;   // the gap needs plain k-NN
    // one launch with the list size of the largest k (a batch mixing k = 10
    // and k = 16 clouds was measured slower with a launch per list size:
    // 16.8 against 14.0 ms for the 256-pair batch's normals)
    timer_search_begin(s);
    if (k_max <= 4) launch_normals<4>(g, xyz, k_max, kc, cap2, min_pts, vp, on, oc, srt, s);
    else if (k_max <= 8) launch_normals<8>(g, xyz, k_max, kc, cap2, min_pts, vp, on, oc, srt, s);
    else if (k_max <= 16) launch_normals<16>(g, xyz, k_max, kc, cap2, min_pts, vp, on, oc, srt, s);
    else launch_normals<32>(g, xyz, k_max, kc, cap2, min_pts, vp, on, oc, srt, s);
    timer_search_end(s);
    return hipGetLastError();
}

hipError_t normals_radius_run(const GridStore &g, float r2, const float *vp, float *on, float *oc, hipStream_t s)
{
    if (g.n <= 0) return hipSuccess;
    int blocks = (int)((g.n + kQThreads - 1) / kQThreads);
    if (g.leaf <= 8) k_normals_radius<8><<<blocks, kQThreads, 0, s>>>(g.view(), g.n, r2, vp[0], vp[1], vp[2], on, oc);
    else if (g.leaf <= 16)
        k_normals_radius<16><<<blocks, kQThreads, 0, s>>>(g.view(), g.n, r2, vp[0], vp[1], vp[2], on, oc);
    else k_normals_radius<32><<<blocks, kQThreads, 0, s>>>(g.view(), g.n, r2, vp[0], vp[1], vp[2], on, oc);
    return hipGetLastError();
}

}  // namespace pcg
