// Point-to-plane ICP on the sparse voxel pyramid of the target.
//
// The loop alternates correspondence search and transform estimation
// (Section 3, "Iterative geometric registration"); correspondences are
// nearest neighbours with a rejection distance and the loop runs a fixed
// number of iterations (Section 4, ICP benchmark); the estimator is the
// linear least-squares point-to-plane method the paper cites (Low 2004).
//
// Per source point (float32): p' = R p + t with the float32 copy of the
// pose, exact nearest target point within d_max (warm-started from the
// previous iteration's match), residual r = (p' - q) . n and Jacobian
// J = [p' x n, n].  The 27 sums of A = sum J^T J (21 unique) and b = J^T r,
// plus sum r^2, are accumulated with compensated float32 arithmetic (TwoSum
// (hi, lo) pairs per lane, merged error-free across the wave and block);
// the inlier count is an integer.  The finalize kernel merges the block
// partials in a fixed order (deterministic), converts to float64 and solves
// the 6x6 system by Cholesky; the increment x = (alpha, beta, gamma, tau) is
// applied as R <- Rz(gamma) Ry(beta) Rx(alpha) R, t <- Rz Ry Rx t + tau in
// float64, and the float32 copy for the next pass is rounded from it.

#include <hip/hip_cooperative_groups.h>

#include "icp.h"
#include "search.h"

namespace cg = cooperative_groups;

namespace pcg {

constexpr int kAcc = 28;            // 21 (A) + 6 (b) + 1 (sum r^2)
constexpr int kIcpMinThreads = 64;  // smallest accumulate block: sizes the workspace

// ICP metrics (Section 3, "Iterative geometric registration": point-to-point
// and point-to-plane metrics and weighted combinations of them)
enum { kMetricPlane = 0, kMetricPoint = 1, kMetricCombined = 2 };
constexpr int kFinThreads = 1024;
constexpr int kGroup = 64;          // block partials merged per k_icp_reduce block

struct IcpState {
    double T[16];          // current pose, float64 row-major
    float Thi[12];         // float32 split of rows of [R | t]: T ~ Thi + Tlo
    float Tlo[12];
    int32_t status;        // PC_ICP_* once stopped, PC_ICP_MAXITER while running
    int32_t iters;         // increments applied
    int32_t stop;          // set once the loop must not continue
    int32_t pad;
    int64_t inliers;       // of the last pass
    double sum_r2;         // of the last pass
};

// one (hi, lo) compensated float32 sum
struct CSum {
    float hi, lo;
};

__device__ inline void two_sum_add(CSum &s, float x)
{
    float t = s.hi + x;
    float bp = t - s.hi;
    float err = (s.hi - (t - bp)) + (x - bp);
    s.hi = t;
    s.lo += err;
}

__device__ inline CSum csum_merge(CSum a, CSum b)
{
    float t = a.hi + b.hi;
    float bp = t - a.hi;
    float err = (a.hi - (t - bp)) + (b.hi - bp);
    CSum r;
    r.hi = t;
    r.lo = (a.lo + b.lo) + err;
    return r;
}

// Correspondence search with a float64 certificate.  The float32 search
// keeps the best candidate and the smallest key of any other candidate; a
// decision (which target point is nearest, whether it is within d_max) is
// taken in float32 only when no float64 evaluation could decide otherwise:
// keys differ from the float64 squared distances of the oracle's
// float64-transformed point by at most err(key), which bounds the rounding
// of the float32 pose, the float32 transform and the key itself.  Ambiguous
// queries (close runners-up or a distance at d_max) are re-decided in
// float64 with the same expressions as the float64 definition.
struct NearBand {
    float bkey;          // best key (float32), and its original index: the
    uint32_t bidx;       // candidate order is (key, index)
    int32_t best_pos;    // sorted position, -1 if none within the cap
    uint32_t best_node;  // node whose scan produced best_pos
    float second;        // smallest key of any other candidate seen
    float delta;         // bound on |p'(float32) - p'(float64)| per axis
    float bnd;           // search radius^2: bkey + 2 err(bkey), updated with bkey

    __device__ void init(float cap2, float dlt)
    {
        delta = dlt;
        bkey = cap2 + err(cap2);
        bidx = 0xffffffffu;
        bnd = bkey + 2.f * err(bkey);
        best_pos = -1;
        best_node = 0xffffffffu;
        second = INFINITY;
    }
    __device__ float err(float key) const
    {
        return 6e-7f * key + 3.5f * delta * sqrtf(key) + 6.f * delta * delta + 1e-30f;
    }
    __device__ float best_key() const { return bkey; }
    __device__ bool have() const { return best_pos >= 0; }
    __device__ float bound2() const { return bnd; }
    __device__ void visit(float qx, float qy, float qz, uint32_t j, const float4 &p, uint32_t m)
    {
        const float key = knn_key(p.x, p.y, p.z, qx, qy, qz);
        const uint32_t idx = __float_as_uint(p.w);
        if (key < bkey || (key == bkey && idx < bidx)) {
            if (best_pos >= 0) second = fminf(second, bkey);
            bkey = key;
            bidx = idx;
            best_pos = (int32_t)j;
            best_node = m;
            bnd = key + 2.f * err(key);
        } else if ((int32_t)j != best_pos) {
            second = fminf(second, key);
        }
    }
};

// float64 re-decision: nearest point by |p' - q|^2 in float64 among those
// with |p' - q|^2 <= d_max^2, ties to the lower original index
struct Near64 {
    double px, py, pz, dmax2, best;
    uint32_t best_orig;
    int32_t best_pos;
    float r2;            // float32 search radius^2 that holds every candidate

    __device__ bool have() const { return true; }
    __device__ float bound2() const { return r2; }
    __device__ void visit(float, float, float, uint32_t j, const float4 &p, uint32_t)
    {
        double dx = px - (double)p.x, dy = py - (double)p.y, dz = pz - (double)p.z;
        double d2 = dx * dx + dy * dy + dz * dz;
        uint32_t o = __float_as_uint(p.w);
        if (d2 <= dmax2 && (d2 < best || (d2 == best && o < best_orig))) {
            best = d2;
            best_orig = o;
            best_pos = (int32_t)j;
        }
    }
};

// p[i] by a load the compiler cannot merge with an earlier load of it, so
// that neither the first value nor what was computed from it is kept in
// registers until this point
__device__ inline float4 reload(const float4 *p, int64_t i)
{
    asm volatile("" : "+s"(p));
    return p[i];
}

// float32 (hi, lo) split of the float64 pose used by the transform below
__device__ inline void split_pose(IcpState *st)
{
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 4; c++) {
            double v = st->T[r * 4 + c];
            float h = (float)v;
            st->Thi[r * 4 + c] = h;
            st->Tlo[r * 4 + c] = (float)(v - (double)h);
        }
}

// One row of p' = R p + t in double-float arithmetic: hi + lo equals the
// product with the float64 pose to about 2^-44 relative.  Products are split
// exactly with fmaf (TwoProd), sums with TwoSum; the lo part of the pose only
// needs plain float32.  This keeps residuals r = (p' - q) . n accurate when
// |p'| is metres and |p' - q| is millimetres.
__device__ inline void df_row(const float *h, const float *l, float px, float py, float pz, float &hi, float &lo)
{
    float a0 = h[0] * px, e0 = __fmaf_rn(h[0], px, -a0);
    float a1 = h[1] * py, e1 = __fmaf_rn(h[1], py, -a1);
    float a2 = h[2] * pz, e2 = __fmaf_rn(h[2], pz, -a2);
    float s0 = h[3] + a0, b0 = s0 - h[3], r0 = (h[3] - (s0 - b0)) + (a0 - b0);
    float s1 = s0 + a1, b1 = s1 - s0, r1 = (s0 - (s1 - b1)) + (a1 - b1);
    float s2 = s1 + a2, b2 = s2 - s1, r2 = (s1 - (s2 - b2)) + (a2 - b2);
    float tail = __fmaf_rn(l[0], px, __fmaf_rn(l[1], py, __fmaf_rn(l[2], pz, l[3])));
    hi = s2;
    lo = ((r0 + r1) + r2) + ((e0 + e1) + e2) + tail;
}

namespace {

// Per pair: pose from init_T (identity when null) and loop state.  A pair
// with no source or no target point starts stopped with NO_INLIERS.
__global__ void k_icp_setup(const double *__restrict__ init_T, const int64_t *__restrict__ soff,
                            const int64_t *__restrict__ toff, const int32_t *__restrict__ max_iters, int np,
                            IcpState *__restrict__ st)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    IcpState *s = st + p;
    for (int i = 0; i < 16; i++) s->T[i] = init_T ? init_T[16 * p + i] : ((i % 5 == 0) ? 1.0 : 0.0);
    split_pose(s);
    bool empty = soff[p + 1] == soff[p] || toff[p + 1] == toff[p];
    s->status = empty ? PC_ICP_NO_INLIERS : PC_ICP_MAXITER;
    s->iters = 0;
    s->stop = (empty || max_iters[p] <= 0) ? 1 : 0;
    s->inliers = 0;
    s->sum_r2 = 0.0;
}

// One pair's layout, written on the device for single-pair calls: source and
// target offsets, blocks and reduction groups, rejection distance and
// iteration limit.
__global__ void k_single_pair(int64_t ns, int64_t nt, int nblk, int ngrp, float dmax, int max_iters,
                              int64_t *__restrict__ soff, int64_t *__restrict__ toff, int32_t *__restrict__ boff,
                              int32_t *__restrict__ goff, float *__restrict__ dm, int32_t *__restrict__ mi)
{
    soff[0] = 0;
    soff[1] = ns;
    toff[0] = 0;
    toff[1] = nt;
    boff[0] = 0;
    boff[1] = nblk;
    goff[0] = 0;
    goff[1] = ngrp;
    dm[0] = dmax;
    mi[0] = max_iters;
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Target normals in sorted order (zero when none are given), with w a lower
// bound of the squared distance from the point to the nearest other point of
// its cloud: 0 when it has an exact duplicate, +inf when it is alone.  No
// other target point can be nearer to anything within half that distance of
// the point.
constexpr int kGapThreads = 256;
__global__ void __launch_bounds__(kGapThreads) k_nrm_gap(GridView g, int64_t n_all, const float *__restrict__ tgt_n,
                                                        float4 *__restrict__ nrm)
{
    __shared__ __align__(8) uint32_t stk[SearchStack::words * kGapThreads];
    const int64_t s = xcd_block(blockIdx.x, gridDim.x) * (int64_t)kGapThreads + threadIdx.x;
    if (s >= n_all) return;
    const GridParams P = g.params[key_cloud(g.keys[s])];
    const float4 p = g.pts[s];
    const uint32_t qi = __float_as_uint(p.w);
    TopK<2> top;
    top.init(2);
    Query q{p.x, p.y, p.z};
    search<TopK<2>, 16>(g, P, q, top, 2, lane_stack<SearchStack>(stk, kGapThreads));
    // the point itself (or an exact duplicate) is first; the second key is
    // the squared distance to the nearest other point, rounded to float32
    // (relative error below 2^-21)
    const float gap = top.h[1] == ~0ull ? INFINITY
                                         : __uint_as_float((uint32_t)(top.h[1] >> 32)) * (1.f - 1.f / (1 << 20));
    float4 o = make_float4(0.f, 0.f, 0.f, gap);
    if (tgt_n) {
        o.x = tgt_n[3 * (int64_t)qi];
        o.y = tgt_n[3 * (int64_t)qi + 1];
        o.z = tgt_n[3 * (int64_t)qi + 2];
    }
    nrm[s] = o;
}

// pair owning block b (or group b) for block offsets off[0..np]
__device__ inline int pair_of(const int32_t *__restrict__ off, int np, int b)
{
    int lo = 0, hi = np - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Correspondences + linearised system.  One source point per lane: the
// search is bound by memory latency, so parallelism comes from many lanes.
// Every block belongs to one pair (its source points, its target cloud and
// its pose).  Each block writes its compensated partial sums; k_icp_reduce
// and the finalize kernel merge them in block order, so the result does not
// depend on scheduling (no atomics, no fences in the hot kernel).
// Block reduction of the 28 per-lane values, error-free in (hi, lo) float
// pairs and in a fixed order: in two passes of 14 sums, every lane stores
// its values in LDS (red: at least 14 * (NT + 1) floats, free on entry),
// then NT / 16 lanes per sum each accumulate 16 of them with TwoSum and
// merge their pairs across those lanes.  Writes part[lblk] and the block's
// inlier count pcnt[lblk].
template <int NT>
__device__ inline void block_partials(const float (&val)[kAcc], uint32_t cnt, float *red, float2 *__restrict__ part,
                                      uint32_t *__restrict__ pcnt, int lblk)
{
    constexpr int kHalf = kAcc / 2;
    constexpr int kRow = NT + 1;                          // padded row (bank spread)
    constexpr int kLanes = NT / 16;
    static_assert(kHalf * kLanes <= NT, "one lane per (sum, share)");
    __shared__ uint32_t wcnt[NT / 64];
    const int tid = threadIdx.x, w = tid >> 6;
    const int ra = tid / kLanes, rk = tid % kLanes;       // sum handled, share
#pragma unroll
    for (int half = 0; half < 2; half++) {
#pragma unroll
        for (int a = 0; a < kHalf; a++) red[a * kRow + tid] = val[half * kHalf + a];
        __syncthreads();
        if (ra < kHalf) {
            CSum c{0.f, 0.f};
#pragma unroll
            for (int k = 0; k < 16; k++) two_sum_add(c, red[ra * kRow + rk + kLanes * k]);
#pragma unroll
            for (int off = kLanes / 2; off > 0; off >>= 1) {
                CSum o{__shfl_xor(c.hi, off), __shfl_xor(c.lo, off)};
                c = csum_merge(c, o);
            }
            if (rk == 0) part[(int64_t)lblk * kAcc + half * kHalf + ra] = make_float2(c.hi, c.lo);
        }
        __syncthreads();
    }
    uint64_t ib = __ballot(cnt != 0);
    if (__lane_id() == 0) wcnt[w] = (uint32_t)__popcll(ib);
    __syncthreads();
    if (tid == 0) {
        uint32_t c = 0;
        for (int x = 0; x < NT / 64; x++) c += wcnt[x];
        pcnt[lblk] = c;
    }
}

// point-to-plane values of one inlier: the 21 upper-triangle entries of
// J^T J, J^T r and r^2 for J = [p' x n, n], r = (p' - q) . n, from the
// double-float p' = (h + l) and the target point t
__device__ inline void plane_values(float hx, float lx, float hy, float ly, float hz, float lz, const float4 &t,
                                    const float4 &n, float (&val)[kAcc])
{
    float qx = hx + lx, qy = hy + ly, qz = hz + lz;
    // residual vector from the double-float p': (hi - q) is exact for
    // nearby points, so it keeps the full accuracy of hi + lo
    float dx = (hx - t.x) + lx, dy = (hy - t.y) + ly, dz = (hz - t.z) + lz;
    float J[6], res;
    res = __fmaf_rn(dz, n.z, __fmaf_rn(dy, n.y, dx * n.x));
    J[0] = __fmaf_rn(qy, n.z, -qz * n.y);
    J[1] = __fmaf_rn(qz, n.x, -qx * n.z);
    J[2] = __fmaf_rn(qx, n.y, -qy * n.x);
    J[3] = n.x;
    J[4] = n.y;
    J[5] = n.z;
    int a = 0;
#pragma unroll
    for (int u = 0; u < 6; u++)
#pragma unroll
        for (int v = u; v < 6; v++) val[a++] = J[u] * J[v];
#pragma unroll
    for (int u = 0; u < 6; u++) val[21 + u] = J[u] * res;
    val[27] = res * res;
}

// The 28 per-point values summed per block, by metric:
//   plane, combined: the 21 upper-triangle entries of A (row-major), the 6
//       of b, the (weighted) squared residual;
//   point: p' - c (3), q - c (3), (p' - c)(q - c)^T (9, row-major),
//       |p' - q|^2, zeros; c = the target cloud's cube centre.
// One accumulate block (block lblk of the pair that owns it): the body of
// k_icp_accum and of the accumulate phase of k_icp_persistent.  stk: the
// block's LDS stack (NearStack::words * NT words), reused for the reduction.
template <int NT, int LEAF, int METRIC>
__device__ inline void accum_block(const GridView &g, const float4 *__restrict__ srcp,
                                   const int64_t *__restrict__ soff, const int32_t *__restrict__ boff, int np,
                                   const float4 *__restrict__ nrm, int2 *__restrict__ prev,
                                   const IcpState *__restrict__ state, const float *__restrict__ dmaxv,
                                   int final_pass, float2 *__restrict__ part, uint32_t *__restrict__ pcnt,
                                   float w_point, float w_plane, int lblk, uint32_t *stk)
{
    const int pr = np > 1 ? pair_of(boff, np, lblk) : 0;
    const IcpState *st = state + pr;
    if (!final_pass && st->stop) return;   // uniform across the block
    const GridParams P = g.params[pr];
    float Rh[12], Rl[12];
#pragma unroll
    for (int i = 0; i < 12; i++) {
        Rh[i] = st->Thi[i];
        Rl[i] = st->Tlo[i];
    }
    const float dmax = dmaxv[pr];
    const double dmax64 = (double)dmax;
    const float dmax2 = dmax * dmax;
    const int64_t i = soff[pr] + (int64_t)(lblk - boff[pr]) * NT + threadIdx.x;
    const bool active = i < soff[pr + 1] && P.n > 0;
    int32_t j = -1;
    float hx = 0.f, lx = 0.f, hy = 0.f, ly = 0.f, hz = 0.f, lz = 0.f;   // double-float p'
    if (active) {
        const float4 sp = srcp[i];
        float px = sp.x, py = sp.y, pz = sp.z;
        df_row(Rh, Rl, px, py, pz, hx, lx);
        df_row(Rh + 4, Rl + 4, px, py, pz, hy, ly);
        df_row(Rh + 8, Rl + 8, px, py, pz, hz, lz);
        // the search needs q alone; the source point and the double-float
        // p' are loaded and computed again after it (registers held across
        // the search cost occupancy, which the search's latency needs)
        Query q{hx + lx, hy + ly, hz + lz};
        // q is p' rounded to float32 (plus ~2^-44 relative): per axis it is
        // within half an ulp, bounded here with slack, of the float64 p'
        float dlt = fmaxf(fmaxf(fabsf(q.x), fabsf(q.y)), fabsf(q.z)) * (1.0f / (1 << 22)) +
                    (fabsf(px) + fabsf(py) + fabsf(pz) + fabsf(Rh[3]) + fabsf(Rh[7]) + fabsf(Rh[11])) *
                        (1.0f / (1 << 30)) + 1e-30f;
        int2 pv = prev[i];          // previous match (sorted position) and its node
        bool done = false;
        NearBand v;
        v.init(dmax2, dlt);
        bool searched = false;
        if (pv.x >= 0) {
            // Previous match q0 (its normal's w: a lower bound of the squared
            // distance from q0 to any other target point of the cloud).  When
            // |p' - q0| is below half that distance, q0 is strictly the
            // nearest target point: no search.
            const float4 p0 = g.pts[pv.x];
            const float4 n0 = nrm[pv.x];
            v.visit(q.x, q.y, q.z, (uint32_t)pv.x, p0, (uint32_t)pv.y);
            if (v.best_pos >= 0) {
                const float u = v.best_key() + v.err(v.best_key());   // >= the float64 |p' - q0|^2
                if (u < dmax2 * (1.0f - 1.0f / (1 << 22)) && 4.f * u * (1.f + 1.f / (1 << 20)) < n0.w) {
                    j = pv.x;
                    done = true;
                } else {
                    const Node nm = g.node[pv.y];
                    searched = search_in_node(g, P, q, v, (uint32_t)pv.y, nm, p0);
                }
            }
        }
        if (!done) {
            if (!searched) search<NearBand, LEAF>(g, P, q, v, 1, lane_stack<NearStack>(stk, NT));
            if (v.best_pos >= 0) {
                float b = v.best_key();
                float e = v.err(b);
                bool sure_in = b + e < dmax2 * (1.0f - 1.0f / (1 << 22));
                bool sure_out = b - e > dmax2 * (1.0f + 1.0f / (1 << 22));
                bool sure_nn = v.second > b + 2.f * e;
                if (sure_nn && sure_in) {
                    j = v.best_pos;
                } else if (!sure_out) {
                    const double *T = st->T;
                    const float4 sp2 = reload(srcp, i);
                    px = sp2.x;
                    py = sp2.y;
                    pz = sp2.z;
                    Near64 w;
                    w.px = T[0] * (double)px + T[1] * (double)py + T[2] * (double)pz + T[3];
                    w.py = T[4] * (double)px + T[5] * (double)py + T[6] * (double)pz + T[7];
                    w.pz = T[8] * (double)px + T[9] * (double)py + T[10] * (double)pz + T[11];
                    w.dmax2 = dmax64 * dmax64;
                    w.best = INFINITY;
                    w.best_orig = 0xffffffffu;
                    w.best_pos = -1;
                    w.r2 = b + 2.f * e;
                    cover<Near64, LEAF>(g, P, q, w, lane_stack<NearStack>(stk, NT), 0u, 0u);
                    j = w.best_pos;
                }
            }
            const int2 pn = v.best_pos >= 0 ? make_int2(v.best_pos, (int32_t)v.best_node) : make_int2(-1, -1);
            if (pn.x != pv.x || pn.y != pv.y) prev[i] = pn;
        }
    }
    if (j >= 0) {
        const float4 sp = reload(srcp, i);
        df_row(Rh, Rl, sp.x, sp.y, sp.z, hx, lx);
        df_row(Rh + 4, Rl + 4, sp.x, sp.y, sp.z, hy, ly);
        df_row(Rh + 8, Rl + 8, sp.x, sp.y, sp.z, hz, lz);
    }
    // This lane's values of the sums (zero when it is not an inlier).
    float val[kAcc];
#pragma unroll
    for (int a = 0; a < kAcc; a++) val[a] = 0.f;
    uint32_t cnt = 0;
    if (j >= 0) {
        float4 n = make_float4(0.f, 0.f, 0.f, 0.f);
        bool use = true;
        const bool need_n = METRIC == kMetricPlane || (METRIC == kMetricCombined && w_plane > 0.f);
        if (need_n) {
            n = nrm[j];
            use = n.x != 0.f || n.y != 0.f || n.z != 0.f;
        }
        if (use) {
            const float4 t = g.pts[j];
            float qx = hx + lx, qy = hy + ly, qz = hz + lz;
            // residual vector from the double-float p': (hi - q) is exact for
            // nearby points, so it keeps the full accuracy of hi + lo
            float dx = (hx - t.x) + lx, dy = (hy - t.y) + ly, dz = (hz - t.z) + lz;
            cnt = 1;
            if (METRIC == kMetricPoint) {
                // offsets from the cube centre keep the cross-covariance sums
                // well conditioned
                const float half = 0.5f * (float)(1u << kBits) * P.h0;
                const float cx = P.ox + half, cy = P.oy + half, cz = P.oz + half;
                float px = (hx - cx) + lx, py = (hy - cy) + ly, pz = (hz - cz) + lz;
                float tx = t.x - cx, ty = t.y - cy, tz = t.z - cz;
                val[0] = px; val[1] = py; val[2] = pz;
                val[3] = tx; val[4] = ty; val[5] = tz;
                val[6] = px * tx; val[7] = px * ty; val[8] = px * tz;
                val[9] = py * tx; val[10] = py * ty; val[11] = py * tz;
                val[12] = pz * tx; val[13] = pz * ty; val[14] = pz * tz;
                val[15] = __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, dx * dx));
            } else {
                plane_values(hx, lx, hy, ly, hz, lz, t, n, val);
                if (METRIC == kMetricCombined) {
                    // point-to-point part: J = [-[p']_x, I], r = p' - q, so
                    // J^T J = [[|p'|^2 I - p' p'^T, [p']_x], [-[p']_x, I]] and
                    // J^T r = [p' x r; r]
                    float Apt[21] = {qy * qy + qz * qz, -qx * qy, -qx * qz, 0.f, -qz, qy,
                                     qx * qx + qz * qz, -qy * qz, qz, 0.f, -qx,
                                     qx * qx + qy * qy, -qy, qx, 0.f,
                                     1.f, 0.f, 0.f,
                                     1.f, 0.f,
                                     1.f};
                    float bpt[6] = {__fmaf_rn(qy, dz, -qz * dy), __fmaf_rn(qz, dx, -qx * dz),
                                    __fmaf_rn(qx, dy, -qy * dx), dx, dy, dz};
#pragma unroll
                    for (int k = 0; k < 21; k++) val[k] = __fmaf_rn(w_point, Apt[k], w_plane * val[k]);
#pragma unroll
                    for (int k = 0; k < 6; k++) val[21 + k] = __fmaf_rn(w_point, bpt[k], w_plane * val[21 + k]);
                    val[27] = __fmaf_rn(w_point, __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, dx * dx)), w_plane * val[27]);
                }
            }
        }
    }
    __syncthreads();                                      // stack no longer in use
    block_partials<NT>(val, cnt, reinterpret_cast<float *>(stk), part, pcnt, lblk);
}

template <int NT, int LEAF, int METRIC>
__global__ void __launch_bounds__(NT)
k_icp_accum(GridView g, const float4 *__restrict__ srcp, const int64_t *__restrict__ soff,
            const int32_t *__restrict__ boff, int np, const float4 *__restrict__ nrm, int2 *__restrict__ prev,
            const IcpState *__restrict__ state, const float *__restrict__ dmaxv, int final_pass,
            float2 *__restrict__ part, uint32_t *__restrict__ pcnt, int nblk, float w_point, float w_plane)
{
    // the DFS stack and, after the search, the reduction buffer share LDS
    static_assert((kAcc / 2) * (NT + 1) <= NearStack::words * NT, "reduction buffer must fit in the stack");
    __shared__ __align__(8) uint32_t stk[NearStack::words * NT];
    accum_block<NT, LEAF, METRIC>(g, srcp, soff, boff, np, nrm, prev, state, dmaxv, final_pass, part, pcnt, w_point,
                                  w_plane, xcd_block(blockIdx.x, nblk), stk);
}

// Projective correspondences (the organized-target association of
// Section 3): p' = T p in float64 (the pose's float64 rows, left to right),
// pixel (floor(u + 0.5), floor(v + 0.5)) of u = fx * p'x / p'z + cx,
// v = fy * p'y / p'z + cy when p'z > 0; an inlier when the pixel is in the
// image and valid (finite, z > 0), its normal is nonzero and
// |p' - q|^2 <= d_max^2 (float64).  The values summed are the point-to-plane
// ones.  No search: one gather of the pixel's point and normal per point.
template <int NT>
__global__ void __launch_bounds__(NT)
k_icp_accum_proj(const float *__restrict__ src, const int64_t *__restrict__ soff, const int32_t *__restrict__ boff,
                 int np, const float *__restrict__ tgt, const float *__restrict__ tnrm, int W, int H, float fx,
                 float fy, float cx, float cy, const IcpState *__restrict__ state, const float *__restrict__ dmaxv,
                 int final_pass, float2 *__restrict__ part, uint32_t *__restrict__ pcnt, int nblk)
{
    __shared__ float red[(kAcc / 2) * (NT + 1)];
    const int lblk = xcd_block(blockIdx.x, nblk);
    const int pr = np > 1 ? pair_of(boff, np, lblk) : 0;
    const IcpState *st = state + pr;
    if (!final_pass && st->stop) return;   // uniform across the block
    const double dmax64 = (double)dmaxv[pr];
    const int64_t i = soff[pr] + (int64_t)(lblk - boff[pr]) * NT + threadIdx.x;
    float val[kAcc];
#pragma unroll
    for (int a = 0; a < kAcc; a++) val[a] = 0.f;
    uint32_t cnt = 0;
    if (i < soff[pr + 1]) {
        const double *T = st->T;
        const double sx = src[3 * i], sy = src[3 * i + 1], sz = src[3 * i + 2];
        const double px = T[0] * sx + T[1] * sy + T[2] * sz + T[3];
        const double py = T[4] * sx + T[5] * sy + T[6] * sz + T[7];
        const double pz = T[8] * sx + T[9] * sy + T[10] * sz + T[11];
        if (pz > 0.0) {
            const double u = (double)fx * px / pz + (double)cx;
            const double v = (double)fy * py / pz + (double)cy;
            const double fu = floor(u + 0.5), fv = floor(v + 0.5);
            if (fu >= 0.0 && fu < (double)W && fv >= 0.0 && fv < (double)H) {
                const int64_t k = (int64_t)fv * W + (int64_t)fu;
                const float4 q = make_float4(tgt[3 * k], tgt[3 * k + 1], tgt[3 * k + 2], 0.f);
                const float4 n = make_float4(tnrm[3 * k], tnrm[3 * k + 1], tnrm[3 * k + 2], 0.f);
                const bool valid = isfinite(q.x) && isfinite(q.y) && isfinite(q.z) && q.z > 0.f;
                const bool has_n = n.x != 0.f || n.y != 0.f || n.z != 0.f;
                const double dx = px - q.x, dy = py - q.y, dz = pz - q.z;
                if (valid && has_n && !(dx * dx + dy * dy + dz * dz > dmax64 * dmax64)) {
                    const float hx = (float)px, hy = (float)py, hz = (float)pz;
                    plane_values(hx, (float)(px - (double)hx), hy, (float)(py - (double)hy), hz,
                                 (float)(pz - (double)hz), q, n, val);
                    cnt = 1;
                }
            }
        }
    }
    block_partials<NT>(val, cnt, red, part, pcnt, lblk);
}

// Merges 32-lane groups of (hi, lo) pairs: lane j of each 32-lane half-wave
// holds one pair; a fixed xor tree leaves the total in lane 0.
__device__ inline CSum merge32(CSum c)
{
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) {
        CSum o{__shfl_xor(c.hi, off), __shfl_xor(c.lo, off)};
        c = csum_merge(c, o);
    }
    return c;
}

__device__ inline uint32_t sum32(uint32_t c)
{
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) c += __shfl_xor(c, off);
    return c;
}

// Merges the partials of up to kGroup (64) consecutive blocks of one pair:
// sum a (thread t >> 5) is loaded by 32 lanes, two partials each, and merged
// by a fixed tree, so the result depends only on the block order.
// Group grp of the pair that owns it, with nthr threads (a multiple of 32:
// every 32-lane group takes the same sums, so its shuffles stay together).
__device__ inline void reduce_group(const float2 *__restrict__ part, const uint32_t *__restrict__ pcnt,
                                    const int32_t *__restrict__ boff, const int32_t *__restrict__ goff, int np,
                                    const IcpState *__restrict__ state, int final_pass, float2 *__restrict__ gpart,
                                    uint32_t *__restrict__ gcnt, int grp, int nthr)
{
    static_assert(kGroup == 64, "two partials per lane of a 32-lane group");
    const int pr = np > 1 ? pair_of(goff, np, grp) : 0;
    if (!final_pass && state[pr].stop) return;
    const int b0 = boff[pr] + (grp - goff[pr]) * kGroup;
    const int gsz = (boff[pr + 1] - b0) < kGroup ? (boff[pr + 1] - b0) : kGroup;
    for (int t = threadIdx.x; t < 32 * (kAcc + 1); t += nthr) {
    const int a = t >> 5, j = t & 31;
    if (a < kAcc) {
        CSum c{0.f, 0.f};
        if (j < gsz) {
            float2 v = part[(int64_t)(b0 + j) * kAcc + a];
            c = CSum{v.x, v.y};
        }
        if (j + 32 < gsz) {
            float2 v = part[(int64_t)(b0 + j + 32) * kAcc + a];
            c = csum_merge(c, CSum{v.x, v.y});
        }
        c = merge32(c);
        if (j == 0) gpart[(int64_t)grp * kAcc + a] = make_float2(c.hi, c.lo);
    } else if (a == kAcc) {
        uint32_t c = (j < gsz ? pcnt[b0 + j] : 0u) + (j + 32 < gsz ? pcnt[b0 + j + 32] : 0u);
        c = sum32(c);
        if (j == 0) gcnt[grp] = c;
    }
    }
}

__global__ void __launch_bounds__(1024) k_icp_reduce(const float2 *__restrict__ part, const uint32_t *__restrict__ pcnt,
                                                   const int32_t *__restrict__ boff, const int32_t *__restrict__ goff,
                                                   int np, const IcpState *__restrict__ state, int final_pass,
                                                   float2 *__restrict__ gpart, uint32_t *__restrict__ gcnt)
{
    reduce_group(part, pcnt, boff, goff, np, state, final_pass, gpart, gcnt, blockIdx.x, blockDim.x);
}

// FP64 Cholesky of the 6x6 SPD A (lower, in place); false when a pivot is
// not above 1e-14 times the largest diagonal entry
__device__ bool chol6(double A[36])
{
    double dmax = 0;
    for (int i = 0; i < 6; i++) dmax = fmax(dmax, A[i * 7]);
    for (int j = 0; j < 6; j++) {
        double s = A[j * 6 + j];
        for (int k = 0; k < j; k++) s -= A[j * 6 + k] * A[j * 6 + k];
        if (!(s > 1e-14 * dmax)) return false;
        double d = sqrt(s);
        A[j * 6 + j] = d;
        for (int i = j + 1; i < 6; i++) {
            double t = A[i * 6 + j];
            for (int k = 0; k < j; k++) t -= A[i * 6 + k] * A[j * 6 + k];
            A[i * 6 + j] = t / d;
        }
    }
    return true;
}

// Cyclic Jacobi rotations on a symmetric 4x4 (row-major, destroyed): on
// return the diagonal holds the eigenvalues and column c of v the unit
// eigenvector of a[c][c].
__device__ void jacobi4(double a[16], double v[16])
{
    for (int i = 0; i < 16; i++) v[i] = (i % 5 == 0) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 50; sweep++) {
        double off = 0.0, dg = 0.0;
        for (int p = 0; p < 4; p++) {
            dg += a[p * 5] * a[p * 5];
            for (int q = p + 1; q < 4; q++) off += a[p * 4 + q] * a[p * 4 + q];
        }
        if (!(off > 1e-36 * dg)) break;
        for (int p = 0; p < 3; p++)
            for (int q = p + 1; q < 4; q++) {
                double apq = a[p * 4 + q];
                if (apq == 0.0) continue;
                double th = (a[q * 5] - a[p * 5]) / (2.0 * apq);
                double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
                for (int r = 0; r < 4; r++) {
                    double x = a[r * 4 + p], y = a[r * 4 + q];
                    a[r * 4 + p] = c * x - sn * y;
                    a[r * 4 + q] = sn * x + c * y;
                }
                for (int r = 0; r < 4; r++) {
                    double x = a[p * 4 + r], y = a[q * 4 + r];
                    a[p * 4 + r] = c * x - sn * y;
                    a[q * 4 + r] = sn * x + c * y;
                }
                a[p * 4 + q] = a[q * 4 + p] = 0.0;
                for (int r = 0; r < 4; r++) {
                    double x = v[r * 4 + p], y = v[r * 4 + q];
                    v[r * 4 + p] = c * x - sn * y;
                    v[r * 4 + q] = sn * x + c * y;
                }
            }
    }
}

// Rotation best aligning p - pbar to q - qbar for the cross-covariance
// H[a][b] = sum (p - pbar)_a (q - qbar)_b, by Horn's (1987) unit-quaternion
// method: the eigenvector of the largest eigenvalue of his symmetric 4x4
// matrix.  *top is that eigenvalue and *gap its distance to the next one
// (the rotation is unique when the gap is positive); q4 = (w, x, y, z).
__device__ void horn_rotation(const double H[9], double dR[9], double *top, double *gap, double q4[4])
{
    const double Sxx = H[0], Sxy = H[1], Sxz = H[2], Syx = H[3], Syy = H[4], Syz = H[5], Szx = H[6], Szy = H[7],
                 Szz = H[8];
    double N[16] = {Sxx + Syy + Szz, Syz - Szy,       Szx - Sxz,        Sxy - Syx,
                    Syz - Szy,       Sxx - Syy - Szz, Sxy + Syx,        Szx + Sxz,
                    Szx - Sxz,       Sxy + Syx,       -Sxx + Syy - Szz, Syz + Szy,
                    Sxy - Syx,       Szx + Sxz,       Syz + Szy,        -Sxx - Syy + Szz};
    double V[16];
    jacobi4(N, V);
    int i1 = 0;
    for (int c = 1; c < 4; c++)
        if (N[c * 5] > N[i1 * 5]) i1 = c;
    double second = -INFINITY;
    for (int c = 0; c < 4; c++)
        if (c != i1) second = fmax(second, N[c * 5]);
    *top = N[i1 * 5];
    *gap = N[i1 * 5] - second;
    double w = V[i1], x = V[4 + i1], y = V[8 + i1], z = V[12 + i1];
    double nq = sqrt(w * w + x * x + y * y + z * z);
    w /= nq; x /= nq; y /= nq; z /= nq;
    if (w < 0.0) { w = -w; x = -x; y = -y; z = -z; }
    q4[0] = w; q4[1] = x; q4[2] = y; q4[3] = z;
    dR[0] = w * w + x * x - y * y - z * z;
    dR[1] = 2.0 * (x * y - w * z);
    dR[2] = 2.0 * (x * z + w * y);
    dR[3] = 2.0 * (x * y + w * z);
    dR[4] = w * w - x * x + y * y - z * z;
    dR[5] = 2.0 * (y * z - w * x);
    dR[6] = 2.0 * (x * z - w * y);
    dR[7] = 2.0 * (y * z + w * x);
    dR[8] = w * w - x * x - y * y + z * z;
}

// One block per pair: merges the pair's group partials in a fixed order;
// iteration: solve and update the pose; final pass: publish pose and
// statistics.
// Solve and update of pair pr from its merged sums (one thread).
__device__ __forceinline__ void finalize_solve(const float2 *red, uint32_t redc, int pr, IcpState *st,
                               const int32_t *__restrict__ max_iters, int final_pass, double conv_tol,
                               double *__restrict__ out_T, pc_icp_stats *out_stats, double *__restrict__ hist,
                               int hist_stride, int metric, const GridParams *__restrict__ params);

// Pair pr: merges its group partials in a fixed order (nthr threads, a
// multiple of 32), then one thread solves (iteration) or publishes the pose
// and statistics (final pass).
__device__ inline void finalize_pair(const float2 *__restrict__ gpart, const uint32_t *__restrict__ gcnt,
                                     const int32_t *__restrict__ goff, IcpState *state,
                                     const int32_t *__restrict__ max_iters, int final_pass, double conv_tol,
                                     double *__restrict__ out_T, pc_icp_stats *out_stats, double *__restrict__ hist,
                                     int hist_stride, int metric, const GridParams *__restrict__ params, int pr,
                                     int nthr)
{
    __shared__ float2 red[32];
    __shared__ uint32_t redc;
    IcpState *st = state + pr;
    if (!final_pass && st->stop) return;
    const int g0 = goff[pr], g1 = goff[pr + 1];
    // sum a (thread t >> 5) over the groups: lane j merges groups j, j+32, ...
    // in order, then a fixed 32-lane tree merges the lanes
    for (int t = threadIdx.x; t < 32 * (kAcc + 1); t += nthr) {
    const int a = t >> 5, j = t & 31;
    if (a < kAcc) {
        CSum c{0.f, 0.f};
        for (int b = g0 + j; b < g1; b += 32) {
            float2 v = gpart[(int64_t)b * kAcc + a];
            c = csum_merge(c, CSum{v.x, v.y});
        }
        c = merge32(c);
        if (j == 0) red[a] = make_float2(c.hi, c.lo);
    } else if (a == kAcc) {
        uint32_t c = 0;
        for (int b = g0 + j; b < g1; b += 32) c += gcnt[b];
        c = sum32(c);
        if (j == 0) redc = c;
    }
    }
    __syncthreads();
    if (threadIdx.x == 0)
        finalize_solve(red, redc, pr, st, max_iters, final_pass, conv_tol, out_T, out_stats, hist, hist_stride, metric,
                       params);
    __syncthreads();   // red is reused by the next pair of this block
}

// With fuse (pairs of at most kFuseGroups groups), the group partials are
// formed here from the block partials, exactly as k_icp_reduce forms them
// (the same loads, merge tree and order), and the reduce launch is skipped.
constexpr int kFuseGroups = 4;
__global__ void __launch_bounds__(kFinThreads) k_icp_finalize(const float2 *__restrict__ gpart,
                                                            const uint32_t *__restrict__ gcnt,
                                                            const int32_t *__restrict__ goff,
                                                            IcpState *state, const int32_t *__restrict__ max_iters,
                                                            int final_pass, double conv_tol,
                                                            double *__restrict__ out_T, pc_icp_stats *out_stats,
                                                            double *__restrict__ hist, int hist_stride, int metric,
                                                            const GridParams *__restrict__ params, int fuse,
                                                            const float2 *__restrict__ part,
                                                            const uint32_t *__restrict__ pcnt,
                                                            const int32_t *__restrict__ boff)
{
    // the merge of finalize_pair with one thread per (sum, lane), and the
    // other waves leave before the solve
    __shared__ float2 red[32];
    __shared__ uint32_t redc;
    const int pr = blockIdx.x;
    IcpState *st = state + pr;
    if (!final_pass && st->stop) return;
    const int g0 = goff[pr], g1 = goff[pr + 1];
    const int a = threadIdx.x >> 5, j = threadIdx.x & 31;
    if (a < kAcc) {
        CSum c{0.f, 0.f};
        if (fuse) {
            // group b's partial (lane 0 of its 32-lane merge, as
            // k_icp_reduce stores it), taken by lane (b - g0) mod 32
            const int bend = boff[pr + 1];
            for (int b = g0; b < g1; b++) {
                const int b0 = boff[pr] + (b - g0) * kGroup;
                const int gsz = (bend - b0) < kGroup ? (bend - b0) : kGroup;
                CSum x{0.f, 0.f};
                if (j < gsz) {
                    float2 v = part[(int64_t)(b0 + j) * kAcc + a];
                    x = CSum{v.x, v.y};
                }
                if (j + 32 < gsz) {
                    float2 v = part[(int64_t)(b0 + j + 32) * kAcc + a];
                    x = csum_merge(x, CSum{v.x, v.y});
                }
                x = merge32(x);
                const int l0 = __lane_id() & 32;   // lane 0 of this 32-lane half
                x = CSum{__shfl(x.hi, l0), __shfl(x.lo, l0)};
                if (((b - g0) & 31) == j) c = csum_merge(c, x);
            }
        } else {
#pragma unroll 4
            for (int b = g0 + j; b < g1; b += 32) {
                float2 v = gpart[(int64_t)b * kAcc + a];
                c = csum_merge(c, CSum{v.x, v.y});
            }
        }
        c = merge32(c);
        if (j == 0) red[a] = make_float2(c.hi, c.lo);
    } else if (a == kAcc) {
        uint32_t c = 0;
        if (fuse) {
            const int bend = boff[pr + 1];
            for (int b = g0; b < g1; b++) {
                const int b0 = boff[pr] + (b - g0) * kGroup;
                const int gsz = (bend - b0) < kGroup ? (bend - b0) : kGroup;
                uint32_t x = (j < gsz ? pcnt[b0 + j] : 0u) + (j + 32 < gsz ? pcnt[b0 + j + 32] : 0u);
                x = sum32(x);
                if (((b - g0) & 31) == j) c += x;
            }
        } else {
            for (int b = g0 + j; b < g1; b += 32) c += gcnt[b];
        }
        c = sum32(c);
        if (j == 0) redc = c;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    finalize_solve(red, redc, pr, st, max_iters, final_pass, conv_tol, out_T, out_stats, hist, hist_stride, metric,
                   params);
}

// Persistent form of the whole loop (point-to-plane, nearest-neighbour
// correspondences): one cooperative launch whose workgroups stay resident
// for every pass.  A pass is the accumulate phase over the block tiles of
// every pair, the group merges and the per-pair solves, separated by grid
// barriers; each phase runs the same device code, on the same blocks,
// groups and pairs, as the lockstep kernels, so results are bit-identical.
// Tiles come from a queue per pass (a counter per pass, zero at launch): a
// workgroup takes the next tile when it has finished its last one, so the
// uneven tile costs even out.  Every workgroup reaches every barrier (loops
// over tiles, groups and pairs may be empty).
template <int NT, int LEAF>
__global__ void __launch_bounds__(NT)
k_icp_persistent(GridView g, const float4 *__restrict__ srcp, const int64_t *__restrict__ soff,
                 const int32_t *__restrict__ boff, const int32_t *__restrict__ goff, int np,
                 const float4 *__restrict__ nrm, int2 *__restrict__ prev, IcpState *state,
                 const float *__restrict__ dmaxv, float2 *__restrict__ part, uint32_t *__restrict__ pcnt,
                 float2 *__restrict__ gpart, uint32_t *__restrict__ gcnt, int nblk, int ngrp, int passes,
                 const int32_t *__restrict__ max_iters, double conv_tol, double *__restrict__ out_T,
                 pc_icp_stats *out_stats, double *__restrict__ hist, int hist_stride,
                 const GridParams *__restrict__ params, int32_t *__restrict__ queue)
{
    static_assert((kAcc / 2) * (NT + 1) <= NearStack::words * NT, "reduction buffer must fit in the stack");
    __shared__ __align__(8) uint32_t stk[NearStack::words * NT];
    __shared__ int next;
    cg::grid_group grid = cg::this_grid();
    const int G = (int)gridDim.x;
    for (int pass = 0; pass < passes; pass++) {
        const int fin = pass == passes - 1;   // the last pass gives the statistics
        for (;;) {
            if (threadIdx.x == 0) next = atomicAdd(queue + pass, 1);
            __syncthreads();
            const int t = next;
            __syncthreads();                  // every lane has read it before it is overwritten
            if (t >= nblk) break;
            accum_block<NT, LEAF, kMetricPlane>(g, srcp, soff, boff, np, nrm, prev, state, dmaxv, fin, part, pcnt,
                                                0.f, 1.f, xcd_block(t, nblk), stk);
        }
        grid.sync();
        for (int grp = (int)blockIdx.x; grp < ngrp; grp += G)
            reduce_group(part, pcnt, boff, goff, np, state, fin, gpart, gcnt, grp, NT);
        grid.sync();
        for (int pr = (int)blockIdx.x; pr < np; pr += G)
            finalize_pair(gpart, gcnt, goff, state, max_iters, fin, conv_tol, out_T, out_stats, hist, hist_stride,
                          kMetricPlane, params, pr, NT);
        grid.sync();
    }
}

__device__ __forceinline__ void finalize_solve(const float2 *red, uint32_t redc, int pr, IcpState *st,
                                               const int32_t *__restrict__ max_iters, int final_pass,
                                               double conv_tol, double *__restrict__ out_T,
                                               pc_icp_stats *out_stats, double *__restrict__ hist, int hist_stride,
                                               int metric, const GridParams *__restrict__ params)
{
    out_T += 16 * pr;
    if (out_stats) out_stats += pr;
    if (hist) hist += (int64_t)hist_stride * pr;
    double sum[kAcc];
    for (int k = 0; k < kAcc; k++) sum[k] = (double)red[k].x + (double)red[k].y;
    int64_t inl = redc;
    const double r2 = metric == kMetricPoint ? sum[15] : sum[27];
    st->inliers = inl;
    st->sum_r2 = r2;
    if (final_pass) {
        for (int i = 0; i < 16; i++) out_T[i] = st->T[i];
        if (out_stats) {
            pc_icp_stats o;
            o.status = st->status;
            o.iterations_run = st->iters;
            o.inliers = inl;
            o.rms = inl > 0 ? sqrt(r2 / (double)inl) : 0.0;
            *out_stats = o;
        }
        return;
    }
    if (inl == 0) {
        st->status = PC_ICP_NO_INLIERS;
        st->stop = 1;
        return;
    }
    if (metric == kMetricPoint) {
        // closed-form fit of the inlier pairs (centroids and cross-covariance
        // from the offsets to the cube centre c, as summed)
        const GridParams &P = params[pr];
        const float half = 0.5f * (float)(1u << kBits) * P.h0;
        const double c[3] = {(double)(P.ox + half), (double)(P.oy + half), (double)(P.oz + half)};
        const double n = (double)inl;
        double H[9], pb[3], qb[3];
        for (int u = 0; u < 3; u++) {
            pb[u] = sum[u] / n;
            qb[u] = sum[3 + u] / n;
        }
        for (int u = 0; u < 3; u++)
            for (int v = 0; v < 3; v++) H[u * 3 + v] = sum[6 + u * 3 + v] - sum[u] * sum[3 + v] / n;
        double dR[9], top, gap, q4[4];
        horn_rotation(H, dR, &top, &gap, q4);
        if (inl < 3 || !(gap > 1e-6 * top)) {
            st->status = PC_ICP_DEGENERATE;
            st->stop = 1;
            return;
        }
        double dt[3];
        for (int r = 0; r < 3; r++) {
            double Rp = dR[r * 3] * (c[0] + pb[0]) + dR[r * 3 + 1] * (c[1] + pb[1]) + dR[r * 3 + 2] * (c[2] + pb[2]);
            dt[r] = (c[r] + qb[r]) - Rp;
        }
        double T[16];
        for (int i = 0; i < 16; i++) T[i] = st->T[i];
        for (int r = 0; r < 3; r++) {
            for (int cc = 0; cc < 3; cc++)
                st->T[r * 4 + cc] = dR[r * 3] * T[cc] + dR[r * 3 + 1] * T[4 + cc] + dR[r * 3 + 2] * T[8 + cc];
            st->T[r * 4 + 3] = dR[r * 3] * T[3] + dR[r * 3 + 1] * T[7] + dR[r * 3 + 2] * T[11] + dt[r];
        }
        split_pose(st);
        if (hist) {
            double *h = hist + 8 * st->iters;
            for (int u = 0; u < 3; u++) {
                h[u] = 2.0 * q4[1 + u];
                h[3 + u] = dt[u];
            }
            h[6] = (double)inl;
            h[7] = r2;
        }
        st->iters++;
        if (conv_tol > 0) {
            double m = 0;
            for (int r = 0; r < 3; r++) {
                for (int cc = 0; cc < 3; cc++) m = fmax(m, fabs(dR[r * 3 + cc] - (r == cc ? 1.0 : 0.0)));
                m = fmax(m, fabs(dt[r]));
            }
            if (m < conv_tol) {
                st->status = PC_ICP_CONVERGED;
                st->stop = 1;
            }
        }
        if (!st->stop && st->iters >= max_iters[pr]) st->stop = 1;
        return;
    }
    double A[36], bv[6];
    int k = 0;
    for (int u = 0; u < 6; u++)
        for (int v = u; v < 6; v++) {
            A[u * 6 + v] = sum[k];
            A[v * 6 + u] = sum[k];
            k++;
        }
    for (int u = 0; u < 6; u++) bv[u] = sum[21 + u];
    if (inl < 6 || !chol6(A)) {
        st->status = PC_ICP_DEGENERATE;
        st->stop = 1;
        return;
    }
    // x = -A^{-1} b with the Cholesky factor
    double y[6], x[6];
    for (int i = 0; i < 6; i++) {
        double v = -bv[i];
        for (int j = 0; j < i; j++) v -= A[i * 6 + j] * y[j];
        y[i] = v / A[i * 6 + i];
    }
    for (int i = 5; i >= 0; i--) {
        double v = y[i];
        for (int j = i + 1; j < 6; j++) v -= A[j * 6 + i] * x[j];
        x[i] = v / A[i * 6 + i];
    }
    double ca = cos(x[0]), sa = sin(x[0]), cb = cos(x[1]), sb = sin(x[1]), cg = cos(x[2]), sg = sin(x[2]);
    // Rz(g) Ry(b) Rx(a)
    double dR[9] = {cg * cb, cg * sb * sa - sg * ca, cg * sb * ca + sg * sa,
                    sg * cb, sg * sb * sa + cg * ca, sg * sb * ca - cg * sa,
                    -sb,     cb * sa,                cb * ca};
    double T[16];
    for (int i = 0; i < 16; i++) T[i] = st->T[i];
    for (int r = 0; r < 3; r++) {
        for (int cc = 0; cc < 3; cc++)
            st->T[r * 4 + cc] = dR[r * 3] * T[cc] + dR[r * 3 + 1] * T[4 + cc] + dR[r * 3 + 2] * T[8 + cc];
        st->T[r * 4 + 3] = dR[r * 3] * T[3] + dR[r * 3 + 1] * T[7] + dR[r * 3 + 2] * T[11] + x[3 + r];
    }
    st->T[12] = st->T[13] = st->T[14] = 0.0;
    st->T[15] = 1.0;
    split_pose(st);
    if (hist) {
        double *h = hist + 8 * st->iters;
        for (int i = 0; i < 6; i++) h[i] = x[i];
        h[6] = (double)inl;
        h[7] = sum[27];
    }
    st->iters++;
    if (conv_tol > 0) {
        double m = 0;
        for (int i = 0; i < 6; i++) m = fmax(m, fabs(x[i]));
        if (m < conv_tol) {
            st->status = PC_ICP_CONVERGED;
            st->stop = 1;
        }
    }
    if (!st->stop && st->iters >= max_iters[pr]) st->stop = 1;   // status stays MAXITER
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
// optional event timer around the iteration kernels (diagnostics)
static hipEvent_t *g_tbeg = nullptr, *g_tend = nullptr;
static int g_tcap = 0, g_tcount = 0;

void icp_set_timer(hipEvent_t *b, hipEvent_t *e, int cap)
{
    g_tbeg = b;
    g_tend = e;
    g_tcap = (b && e && cap > 0) ? cap : 0;
    g_tcount = 0;
}

int icp_timer_count() { return g_tcount; }

void timer_slot_begin(int slot, hipStream_t st)
{
    if (slot < g_tcap) (void)hipEventRecord(g_tbeg[slot], st);
}

void timer_slot_end(int slot, hipStream_t st)
{
    if (slot < g_tcap) {
        (void)hipEventRecord(g_tend[slot], st);
        if (g_tcount < slot + 1) g_tcount = slot + 1;
    }
}

// the search kernel of a k-NN or normals call takes slot 0
void timer_search_begin(hipStream_t st) { timer_slot_begin(0, st); }
void timer_search_end(hipStream_t st) { timer_slot_end(0, st); }

void icp_carve(Carver &c, int np, int64_t ns, int64_t nt, int64_t nblk, int64_t ngrp, int iters_max,
               IcpStore &s)
{
    int np1 = np > 0 ? np : 1;
    grid_carve(c, nt, np1, s.grid);
    int64_t nt1 = nt > 0 ? nt : 1, ns1 = ns > 0 ? ns : 1;
    s.np = np1;
    s.nblk = (int)nblk;
    s.ngrp = (int)ngrp;
    s.threads = kIcpMinThreads;
    s.leaf = 16;
    s.metric = kMetricPlane;
    s.w_point = 0.f;
    s.w_plane = 1.f;
    s.assoc = kAssocNearest;
    s.ptgt = s.pnrm = nullptr;
    s.width = s.height = 0;
    s.K[0] = s.K[1] = s.K[2] = s.K[3] = 0.f;
    s.grid_built = false;
    s.nrm_ready = false;
    s.sort_src = true;
    s.persistent = false;
    s.max_pair_groups = 1 << 30;   // unknown: no fused merge
    s.iters_max = iters_max > 0 ? iters_max : 0;
    s.nrm = c.take<float4>(nt1);
    s.prev = c.take<int2>(ns1);
    s.st = c.take<IcpState>(np1);
    s.soff = c.take<int64_t>(np1 + 1);
    s.boff = c.take<int32_t>(np1 + 1);
    s.goff = c.take<int32_t>(np1 + 1);
    s.dmax = c.take<float>(np1);
    s.maxit = c.take<int32_t>(np1);
    grid_carve_sort(c, ns, np1, s.ssrc);
    s.ssrc.off = s.soff;            // the sort splits the sources by pair
    s.part = c.take<float2>((size_t)(nblk > 0 ? nblk : 1) * kAcc);
    s.pcnt = c.take<uint32_t>((size_t)(nblk > 0 ? nblk : 1));
    s.gpart = c.take<float2>((size_t)(ngrp > 0 ? ngrp : 1) * kAcc);
    s.gcnt = c.take<uint32_t>((size_t)(ngrp > 0 ? ngrp : 1));
    s.hist_stride = 8 * (s.iters_max > 0 ? s.iters_max : 1);
    s.hist = c.take<double>((size_t)s.hist_stride * np1);
    s.queue = c.take<int32_t>((size_t)s.iters_max + 1);
}

int64_t icp_blocks(int64_t ns, int threads) { return (ns + threads - 1) / threads; }
int64_t icp_blocks_max(int64_t ns) { return icp_blocks(ns, kIcpMinThreads); }
int64_t icp_groups(int64_t nblk) { return (nblk + kGroup - 1) / kGroup; }

hipError_t icp_layout_single(IcpStore &s, int64_t ns, int64_t nt, float dmax, int max_iters, hipStream_t st)
{
    k_single_pair<<<1, 1, 0, st>>>(ns, nt, s.nblk, s.ngrp, dmax, max_iters, s.soff, s.grid.off, s.boff, s.goff,
                                   s.dmax, s.maxit);
    return hipGetLastError();
}

template <int NT, int LEAF, int M>
static void launch_accum_t(IcpStore &s, const float *src, int fin, hipStream_t st)
{
    k_icp_accum<NT, LEAF, M><<<s.nblk, NT, 0, st>>>(s.grid.view(), s.ssrc.pts, s.soff, s.boff, s.np, s.nrm, s.prev,
                                                    s.st, s.dmax, fin, s.part, s.pcnt, s.nblk, s.w_point,
                                                    s.w_plane);
}

template <int NT, int LEAF>
static void launch_accum_metric(IcpStore &s, const float *src, int fin, hipStream_t st)
{
    if (s.metric == kMetricPoint) launch_accum_t<NT, LEAF, kMetricPoint>(s, src, fin, st);
    else if (s.metric == kMetricCombined) launch_accum_t<NT, LEAF, kMetricCombined>(s, src, fin, st);
    else launch_accum_t<NT, LEAF, kMetricPlane>(s, src, fin, st);
}

template <int NT>
static void launch_accum_leaf(IcpStore &s, const float *src, int fin, hipStream_t st)
{
    if (s.leaf <= 8) launch_accum_metric<NT, 8>(s, src, fin, st);
    else if (s.leaf <= 16) launch_accum_metric<NT, 16>(s, src, fin, st);
    else launch_accum_metric<NT, 32>(s, src, fin, st);
}

template <int NT>
static void launch_accum_proj(IcpStore &s, const float *src, int fin, hipStream_t st)
{
    k_icp_accum_proj<NT><<<s.nblk, NT, 0, st>>>(src, s.soff, s.boff, s.np, s.ptgt, s.pnrm, s.width, s.height, s.K[0],
                                                s.K[1], s.K[2], s.K[3], s.st, s.dmax, fin, s.part, s.pcnt, s.nblk);
}

// The persistent loop as one cooperative launch: as many workgroups as are
// co-resident (a multiple of 8, at most one per tile), all passes inside.
template <int NT, int LEAF>
static hipError_t launch_persistent_t(IcpStore &s, double conv_tol, double *out_T, pc_icp_stats *out_stats,
                                      hipStream_t st)
{
    auto kern = k_icp_persistent<NT, LEAF>;
    int dev = 0, cus = 0, occ = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, NT, 0);
    if (e != hipSuccess) return e;
    int need = s.nblk > s.ngrp ? s.nblk : s.ngrp;
    need = need > s.np ? need : s.np;
    int G = (occ * cus) / 8 * 8;
    const int need8 = (need + 7) / 8 * 8;
    G = G < need8 ? G : need8;
    if (G < 8) return hipErrorLaunchOutOfResources;
    GridView gv = s.grid.view();
    const float4 *srcp = s.ssrc.pts;
    const int64_t *soff = s.soff;
    const int32_t *boff = s.boff, *goff = s.goff, *maxit = s.maxit;
    int np = s.np, nblk = s.nblk, ngrp = s.ngrp, passes = s.iters_max + 1, hist_stride = s.hist_stride;
    const float4 *nrm = s.nrm;
    int2 *prev = s.prev;
    IcpState *state = s.st;
    const float *dmax = s.dmax;
    float2 *part = s.part, *gpart = s.gpart;
    uint32_t *pcnt = s.pcnt, *gcnt = s.gcnt;
    double *hist = s.hist;
    const GridParams *params = s.grid.params;
    int32_t *queue = s.queue;
    // the per-pass tile counters start at zero (a fill kernel: the call stays capturable)
    k_fill_i32<<<1, 256, 0, st>>>(queue, passes, 0);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    void *args[] = {&gv,   &srcp, &soff,  &boff,   &goff,  &np,     &nrm,   &prev,     &state,   &dmax,
                    &part, &pcnt, &gpart, &gcnt,   &nblk,  &ngrp,   &passes, &maxit,   &conv_tol, &out_T,
                    &out_stats, &hist, &hist_stride, &params, &queue};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(kern), dim3(G), dim3(NT), args, 0, st);
}

template <int NT>
static hipError_t launch_persistent_leaf(IcpStore &s, double conv_tol, double *out_T, pc_icp_stats *out_stats,
                                         hipStream_t st)
{
    if (s.leaf <= 8) return launch_persistent_t<NT, 8>(s, conv_tol, out_T, out_stats, st);
    if (s.leaf <= 16) return launch_persistent_t<NT, 16>(s, conv_tol, out_T, out_stats, st);
    return launch_persistent_t<NT, 32>(s, conv_tol, out_T, out_stats, st);
}

static hipError_t launch_persistent(IcpStore &s, double conv_tol, double *out_T, pc_icp_stats *out_stats,
                                    hipStream_t st)
{
    if (s.threads <= 64) return launch_persistent_leaf<64>(s, conv_tol, out_T, out_stats, st);
    if (s.threads <= 128) return launch_persistent_leaf<128>(s, conv_tol, out_T, out_stats, st);
    return launch_persistent_leaf<256>(s, conv_tol, out_T, out_stats, st);
}

static void launch_accum(IcpStore &s, const float *src, int fin, hipStream_t st)
{
    if (s.assoc == kAssocProjective) {
        if (s.threads <= 64) launch_accum_proj<64>(s, src, fin, st);
        else if (s.threads <= 128) launch_accum_proj<128>(s, src, fin, st);
        else launch_accum_proj<256>(s, src, fin, st);
        return;
    }
    if (s.threads <= 64) launch_accum_leaf<64>(s, src, fin, st);
    else if (s.threads <= 128) launch_accum_leaf<128>(s, src, fin, st);
    else launch_accum_leaf<256>(s, src, fin, st);
}

hipError_t icp_run(IcpStore &s, const float *src, int64_t ns, const float *tgt, const float *tgt_n,
                   const double *init_T, double conv_tol, double *out_T, pc_icp_stats *out_stats, hipStream_t st)
{
    const int np = s.np;
    k_icp_setup<<<(np + 63) / 64, 64, 0, st>>>(init_T, s.soff, s.grid.off, s.maxit, np, s.st);
    hipError_t e = hipSuccess;
    if (s.assoc == kAssocNearest) {
        if (!s.grid_built) {
            e = grid_build(s.grid, tgt, st);
            if (e != hipSuccess) return e;
        }
        // queries in Morton order: the lanes of a wave search neighbouring
        // cells in every iteration (a rigid motion keeps them together);
        // otherwise in input order
        e = s.sort_src ? grid_sort_points(s.ssrc, src, st) : grid_pack_points(s.ssrc, src, st);
        if (e != hipSuccess) return e;
        // target normals in sorted order, with the gaps of the match certificate
        if (s.grid.n > 0 && !s.nrm_ready)
            k_nrm_gap<<<(int)((s.grid.n + kGapThreads - 1) / kGapThreads), kGapThreads, 0, st>>>(s.grid.view(),
                                                                                                   s.grid.n, tgt_n,
                                                                                                   s.nrm);
    } else {
        s.ptgt = tgt;
        s.pnrm = tgt_n;
    }
    if (ns > 0) {
        int fb = (int)((2 * ns + 255) / 256 < 2048 ? (2 * ns + 255) / 256 : 2048);
        k_fill_i32<<<fb, 256, 0, st>>>((int32_t *)s.prev, 2 * ns, -1);
    }
    g_tcount = 0;
    if (s.persistent && s.assoc == kAssocNearest && s.metric == kMetricPlane && s.nblk > 0) {
        // the whole loop in one launch; the timer's slot 0 spans it
        if (g_tcap > 0) (void)hipEventRecord(g_tbeg[0], st);
        e = launch_persistent(s, conv_tol, out_T, out_stats, st);
        if (g_tcap > 0) {
            (void)hipEventRecord(g_tend[0], st);
            g_tcount = 1;
        }
        return e != hipSuccess ? e : hipGetLastError();
    }
    // small pairs: the solve kernel merges the block partials itself
    const bool fuse = s.max_pair_groups <= kFuseGroups;
    for (int pass = 0; pass <= s.iters_max; pass++) {
        const int fin = pass == s.iters_max;   // the last pass gives the statistics
        const bool timed = !fin && pass < g_tcap;
        if (s.nblk > 0) {
            if (timed) (void)hipEventRecord(g_tbeg[pass], st);
            launch_accum(s, src, fin, st);
            if (timed) {
                (void)hipEventRecord(g_tend[pass], st);
                g_tcount = pass + 1;
            }
            if (!fuse)
                k_icp_reduce<<<s.ngrp, 1024, 0, st>>>(s.part, s.pcnt, s.boff, s.goff, np, s.st, fin, s.gpart,
                                                      s.gcnt);
        }
        k_icp_finalize<<<np, kFinThreads, 0, st>>>(s.gpart, s.gcnt, s.goff, s.st, s.maxit, fin, conv_tol, out_T,
                                                   out_stats, s.hist, s.hist_stride, s.metric, s.grid.params,
                                                   fuse ? 1 : 0, s.part, s.pcnt, s.boff);
    }
    return hipGetLastError();
}

}  // namespace pcg
