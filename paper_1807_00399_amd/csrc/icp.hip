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

#include "icp.h"
#include "search.h"

namespace pcg {

constexpr int kAcc = 28;            // 21 (A) + 6 (b) + 1 (sum r^2)
constexpr int kIcpThreads = 256;
constexpr int kFinThreads = 1024;

struct IcpState {
    double T[16];          // current pose, float64 row-major
    float Tf[12];          // float32 copy: rows of [R | t]
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

namespace {

__global__ void k_icp_setup(const double *__restrict__ init_T, IcpState *st)
{
    for (int i = 0; i < 16; i++) st->T[i] = init_T ? init_T[i] : ((i % 5 == 0) ? 1.0 : 0.0);
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 4; c++) st->Tf[r * 4 + c] = (float)st->T[r * 4 + c];
    st->status = PC_ICP_MAXITER;
    st->iters = 0;
    st->stop = 0;
    st->inliers = 0;
    st->sum_r2 = 0.0;
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// correspondences + linearised system, partial sums per block
template <int PPT>
__global__ void __launch_bounds__(kIcpThreads) k_icp_accum(GridView g, const float *__restrict__ src, int64_t ns,
                                                         const float4 *__restrict__ nrm,
                                                         int32_t *__restrict__ prev, const IcpState *__restrict__ st,
                                                         float dmax2, int final_pass, float2 *__restrict__ part,
                                                         uint32_t *__restrict__ pcnt)
{
    __shared__ uint2 stk[kStack * kIcpThreads];
    __shared__ float2 wsum[kIcpThreads / 64][kAcc];
    __shared__ uint32_t wcnt[kIcpThreads / 64];
    if (!final_pass && st->stop) return;   // uniform across the grid
    const GridParams P = *g.params;
    float R[12];
#pragma unroll
    for (int i = 0; i < 12; i++) R[i] = st->Tf[i];
    CSum acc[kAcc];
#pragma unroll
    for (int a = 0; a < kAcc; a++) acc[a] = CSum{0.f, 0.f};
    uint32_t cnt = 0;
    int64_t base = (int64_t)blockIdx.x * (kIcpThreads * PPT) + threadIdx.x;
    for (int r = 0; r < PPT; r++) {
        int64_t i = base + (int64_t)r * kIcpThreads;
        if (i >= ns) break;
        float px = src[3 * i], py = src[3 * i + 1], pz = src[3 * i + 2];
        Query q;
        q.x = __fmaf_rn(R[0], px, __fmaf_rn(R[1], py, __fmaf_rn(R[2], pz, R[3])));
        q.y = __fmaf_rn(R[4], px, __fmaf_rn(R[5], py, __fmaf_rn(R[6], pz, R[7])));
        q.z = __fmaf_rn(R[8], px, __fmaf_rn(R[9], py, __fmaf_rn(R[10], pz, R[11])));
        TopK<1> top;
        top.init_capped(dmax2);
        int32_t j0 = prev[i];
        if (j0 >= 0) {
            float4 c = g.pts[j0];
            float key = knn_key(c.x, c.y, c.z, q.x, q.y, q.z);
            top.insert(((uint64_t)__float_as_uint(key) << 32) | __float_as_uint(c.w), j0);
        }
        search<1, 16>(g, P, q, top, 1, dmax2, stk + threadIdx.x, kIcpThreads);
        int32_t j = top.best_pos;
        prev[i] = j;
        if (j < 0) continue;
        float4 n = nrm[j];
        if (n.x == 0.f && n.y == 0.f && n.z == 0.f) continue;
        float4 t = g.pts[j];
        float dx = q.x - t.x, dy = q.y - t.y, dz = q.z - t.z;
        float res = __fmaf_rn(dz, n.z, __fmaf_rn(dy, n.y, dx * n.x));
        float J[6];
        J[0] = __fmaf_rn(q.y, n.z, -q.z * n.y);
        J[1] = __fmaf_rn(q.z, n.x, -q.x * n.z);
        J[2] = __fmaf_rn(q.x, n.y, -q.y * n.x);
        J[3] = n.x;
        J[4] = n.y;
        J[5] = n.z;
        int a = 0;
#pragma unroll
        for (int u = 0; u < 6; u++)
#pragma unroll
            for (int v = u; v < 6; v++) two_sum_add(acc[a++], J[u] * J[v]);
#pragma unroll
        for (int u = 0; u < 6; u++) two_sum_add(acc[21 + u], J[u] * res);
        two_sum_add(acc[27], res * res);
        cnt++;
    }
    // error-free merge across the wave (every lane ends with the same sums)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int a = 0; a < kAcc; a++) {
            CSum o;
            o.hi = __shfl_xor(acc[a].hi, off);
            o.lo = __shfl_xor(acc[a].lo, off);
            acc[a] = csum_merge(acc[a], o);
        }
        cnt += __shfl_xor(cnt, off);
    }
    int w = threadIdx.x >> 6;
    if (__lane_id() == 0) {
#pragma unroll
        for (int a = 0; a < kAcc; a++) wsum[w][a] = make_float2(acc[a].hi, acc[a].lo);
        wcnt[w] = cnt;
    }
    __syncthreads();
    if (threadIdx.x < kAcc) {
        CSum s{0.f, 0.f};
        for (int x = 0; x < kIcpThreads / 64; x++) s = csum_merge(s, CSum{wsum[x][threadIdx.x].x, wsum[x][threadIdx.x].y});
        part[(int64_t)blockIdx.x * kAcc + threadIdx.x] = make_float2(s.hi, s.lo);
    } else if (threadIdx.x == kAcc) {
        uint32_t c = 0;
        for (int x = 0; x < kIcpThreads / 64; x++) c += wcnt[x];
        pcnt[blockIdx.x] = c;
    }
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

// reduces the block partials in a fixed order; iteration: solve and update
// the pose; final pass: publish pose and statistics
__global__ void __launch_bounds__(kFinThreads) k_icp_finalize(const float2 *__restrict__ part,
                                                            const uint32_t *__restrict__ pcnt, int nblk,
                                                            IcpState *st, int final_pass, double conv_tol,
                                                            double *__restrict__ out_T, pc_icp_stats *out_stats,
                                                            double *__restrict__ hist)
{
    constexpr int G = kFinThreads / 32;   // block groups
    __shared__ float2 red[G][32];
    __shared__ uint32_t credg[G];
    if (!final_pass && st->stop) return;
    int t = threadIdx.x, grp = t >> 5, a = t & 31;
    CSum s{0.f, 0.f};
    uint32_t c = 0;
    for (int b = grp; b < nblk; b += G) {
        if (a < kAcc) {
            float2 v = part[(int64_t)b * kAcc + a];
            s = csum_merge(s, CSum{v.x, v.y});
        } else if (a == kAcc) {
            c += pcnt[b];
        }
    }
    red[grp][a] = make_float2(s.hi, s.lo);
    if (a == kAcc) credg[grp] = c;
    __syncthreads();
    if (t != 0) return;
    double sum[kAcc];
    for (int k = 0; k < kAcc; k++) {
        CSum m{0.f, 0.f};
        for (int x = 0; x < G; x++) m = csum_merge(m, CSum{red[x][k].x, red[x][k].y});
        sum[k] = (double)m.hi + (double)m.lo;
    }
    int64_t inl = 0;
    for (int x = 0; x < G; x++) inl += credg[x];
    st->inliers = inl;
    st->sum_r2 = sum[27];
    if (final_pass) {
        for (int i = 0; i < 16; i++) out_T[i] = st->T[i];
        if (out_stats) {
            pc_icp_stats o;
            o.status = st->status;
            o.iterations_run = st->iters;
            o.inliers = inl;
            o.rms = inl > 0 ? sqrt(sum[27] / (double)inl) : 0.0;
            *out_stats = o;
        }
        return;
    }
    if (inl == 0) {
        st->status = PC_ICP_NO_INLIERS;
        st->stop = 1;
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
    for (int r = 0; r < 3; r++)
        for (int cc = 0; cc < 4; cc++) st->Tf[r * 4 + cc] = (float)st->T[r * 4 + cc];
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
}

__global__ void k_icp_empty(const double *__restrict__ init_T, double *out_T, pc_icp_stats *out_stats)
{
    for (int i = 0; i < 16; i++) out_T[i] = init_T ? init_T[i] : ((i % 5 == 0) ? 1.0 : 0.0);
    if (out_stats) {
        pc_icp_stats o;
        o.status = PC_ICP_NO_INLIERS;
        o.iterations_run = 0;
        o.inliers = 0;
        o.rms = 0.0;
        *out_stats = o;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static int icp_ppt(int64_t ns)
{
    int64_t per = (ns + (int64_t)kIcpThreads * 1024 - 1) / ((int64_t)kIcpThreads * 1024);
    if (per <= 1) return 1;
    if (per <= 2) return 2;
    if (per <= 4) return 4;
    if (per <= 8) return 8;
    return 16;
}

void icp_carve(Carver &c, int64_t ns, int64_t nt, int max_iters, IcpStore &s)
{
    grid_carve(c, nt, s.grid);
    int64_t nt1 = nt > 0 ? nt : 1, ns1 = ns > 0 ? ns : 1;
    s.nrm = c.take<float4>(nt1);
    s.prev = c.take<int32_t>(ns1);
    s.st = c.take<IcpState>(1);
    s.ppt = icp_ppt(ns1);
    s.nblk = (int)((ns1 + (int64_t)kIcpThreads * s.ppt - 1) / ((int64_t)kIcpThreads * s.ppt));
    s.part = c.take<float2>((size_t)s.nblk * kAcc);
    s.pcnt = c.take<uint32_t>((size_t)s.nblk);
    s.hist = c.take<double>((size_t)8 * (max_iters > 0 ? max_iters : 1));
}

template <int PPT>
static void launch_accum(IcpStore &s, const float *src, int64_t ns, float dmax2, int final_pass, hipStream_t st)
{
    k_icp_accum<PPT><<<s.nblk, kIcpThreads, 0, st>>>(s.grid.view(), src, ns, s.nrm, s.prev, s.st, dmax2,
                                                     final_pass, s.part, s.pcnt);
}

static void accum(IcpStore &s, const float *src, int64_t ns, float dmax2, int final_pass, hipStream_t st)
{
    switch (s.ppt) {
    case 1: launch_accum<1>(s, src, ns, dmax2, final_pass, st); break;
    case 2: launch_accum<2>(s, src, ns, dmax2, final_pass, st); break;
    case 4: launch_accum<4>(s, src, ns, dmax2, final_pass, st); break;
    case 8: launch_accum<8>(s, src, ns, dmax2, final_pass, st); break;
    default: launch_accum<16>(s, src, ns, dmax2, final_pass, st); break;
    }
}

hipError_t icp_run(IcpStore &s, const float *src, int64_t ns, const float *tgt, const float *tgt_n, int64_t nt,
                   const double *init_T, float dmax, int max_iters, double conv_tol, double *out_T,
                   pc_icp_stats *out_stats, hipStream_t st)
{
    if (ns <= 0 || nt <= 0) {
        k_icp_empty<<<1, 1, 0, st>>>(init_T, out_T, out_stats);
        return hipGetLastError();
    }
    k_icp_setup<<<1, 1, 0, st>>>(init_T, s.st);
    hipError_t e = grid_build(s.grid, tgt, st);
    if (e != hipSuccess) return e;
    e = grid_gather3(s.grid, tgt_n, s.nrm, st);
    if (e != hipSuccess) return e;
    k_fill_i32<<<(int)((ns + 255) / 256 < 2048 ? (ns + 255) / 256 : 2048), 256, 0, st>>>(s.prev, ns, -1);
    float dmax2 = dmax * dmax;
    for (int it = 0; it < max_iters; it++) {
        accum(s, src, ns, dmax2, 0, st);
        k_icp_finalize<<<1, kFinThreads, 0, st>>>(s.part, s.pcnt, s.nblk, s.st, 0, conv_tol, out_T, out_stats,
                                                  s.hist);
    }
    accum(s, src, ns, dmax2, 1, st);
    k_icp_finalize<<<1, kFinThreads, 0, st>>>(s.part, s.pcnt, s.nblk, s.st, 1, conv_tol, out_T, out_stats, s.hist);
    return hipGetLastError();
}

}  // namespace pcg
