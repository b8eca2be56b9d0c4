// Exact nearest-neighbour search over the sparse voxel pyramid.
//
// One lane answers one query.  The traversal is generic over a candidate
// visitor V (the ranking and the running search radius live there):
//   bool  V::have()          a finite radius is already known (warm start)
//   float V::bound2()        current search radius^2 (float32, inclusive)
//   void  V::visit(j, p)     offer sorted point j with coordinates p
//
// The search has two phases:
//   seed  - the smallest cell containing the query that holds `need` points
//           is searched first, which gives a finite radius;
//   cover - the cells of the coarsest useful level (width >= 2R) that meet
//           the ball of radius R are searched depth-first, children nearest
//           first, skipping every cell whose box is farther than the current
//           radius and every point range the seed already contributed.
// Cell boxes are shrunk by an absolute margin and a relative factor, so a
// cell is skipped only when every point in it is strictly outside the
// radius: no candidate inside the radius is ever missed, ties included.
#pragma once

#include "common.h"

namespace pcg {

constexpr int kStack = 16;              // per-lane DFS stack entries (LDS)
constexpr int kVisitBudget = 1 << 20;   // node pops per DFS; only a corrupted tree reaches it

__device__ inline uint64_t enc_cand(float key, float w) { return ((uint64_t)__float_as_uint(key) << 32) | __float_as_uint(w); }

// k best candidates by (float32 key, original index): the k-NN definition.
template <int KT>
struct TopK {
    uint64_t h[KT];     // ascending; ~0 = empty; 0 = padding when k < KT

    __device__ void init(int k)
    {
#pragma unroll
        for (int s = 0; s < KT; s++) h[s] = (s < KT - k) ? 0ull : ~0ull;
    }
    __device__ bool have() const { return h[KT - 1] != ~0ull; }
    __device__ float bound2() const
    {
        return have() ? __uint_as_float((uint32_t)(h[KT - 1] >> 32)) : INFINITY;
    }
    __device__ void insert(uint64_t c)
    {
        if (c < h[KT - 1]) {
#pragma unroll
            for (int s = KT - 1; s > 0; --s) {
                uint64_t prev = h[s - 1];
                uint64_t cur = h[s];
                h[s] = (c < prev) ? prev : ((c < cur) ? c : cur);
            }
            h[0] = (c < h[0]) ? c : h[0];
        }
    }
    __device__ void visit(float qx, float qy, float qz, uint32_t, const float4 &p)
    {
        insert(enc_cand(knn_key(p.x, p.y, p.z, qx, qy, qz), p.w));
    }
};

struct Query {
    float x, y, z;
};

// scan sorted points [s, e) minus the excluded run [xs, xe)
template <class V>
__device__ inline void scan_range(const float4 *__restrict__ pts, uint32_t s, uint32_t e, uint32_t xs,
                                  uint32_t xe, const Query &q, V &v)
{
    uint32_t a0 = s, a1 = e, b0 = e, b1 = e;
    if (xs < xe && xs < e && xe > s) {   // overlap with the excluded run (nested or disjoint)
        a1 = xs > s ? xs : s;
        b0 = xe < e ? xe : e;
    }
    for (uint32_t j = a0; j < a1; j++) v.visit(q.x, q.y, q.z, j, pts[j]);
    for (uint32_t j = b0; j < b1; j++) v.visit(q.x, q.y, q.z, j, pts[j]);
}

// Depth-first search from the entries already on the stack.
// stk: this lane's stack column (stride `stride` entries).
template <class V, int LEAF>
__device__ inline void dfs(const GridView &g, const GridParams &P, const Query &q, V &v, uint2 *stk, int stride,
                           int sp, uint32_t xs, uint32_t xe)
{
    for (int visits = 0; sp > 0 && visits < kVisitBudget; visits++) {
        --sp;
        uint2 e = stk[sp * stride];
        float b2 = v.bound2();
        if (__uint_as_float(e.y) > b2) continue;
        uint32_t m = e.x;
        NodeHdr h = g.hdr[m];
        if (h.start >= xs && h.start + h.count <= xe) continue;      // already searched
        int lvl = g.box[m].level;
        bool leaf = (h.count <= (uint32_t)LEAF) || lvl == P.lmin || sp + (int)h.nchild > kStack;
        if (leaf) {
            scan_range(g.pts, h.start, h.start + h.count, xs, xe, q, v);
            continue;
        }
        // push children: those not containing q first, so the one holding
        // q (mindist 0) is searched next
        for (int pass = 0; pass < 2; pass++) {
            for (uint32_t c = 0; c < h.nchild; c++) {
                uint32_t ch = h.first_child + c;
                NodeBox bx = g.box[ch];
                float d2 = cell_mindist2(P, q.x, q.y, q.z, bx.cx, bx.cy, bx.cz, bx.level);
                bool inside = d2 == 0.f;
                if ((pass == 0) == inside) continue;
                if (d2 > b2) continue;
                stk[sp * stride] = make_uint2(ch, __float_as_uint(d2));
                ++sp;
            }
        }
    }
}

// Cover phase: every cell meeting the ball of the visitor's current radius.
template <class V, int LEAF>
__device__ inline void cover(const GridView &g, const GridParams &P, const Query &q, V &v, uint2 *stk, int stride,
                             uint32_t xs, uint32_t xe)
{
    const float inv = P.inv_h0;
    float b2 = v.bound2();
    if (!(b2 < INFINITY)) return;
    float R = sqrtf(b2) * (1.0f + 1.0f / (1 << 20)) + P.margin;
    // coarsest needed level: cell width >= 2R (with slack) so the ball box
    // meets at most two cells per axis
    int l = P.lmin;
    while (l < kLevels - 1 && P.h0 * (float)(1u << l) * (1.0f - 1.0f / 1024) < 2.0f * R) l++;
    uint32_t lo[3], hi[3];
    lo[0] = cell0(q.x - R, P.ox, inv) >> l;
    hi[0] = cell0(q.x + R, P.ox, inv) >> l;
    lo[1] = cell0(q.y - R, P.oy, inv) >> l;
    hi[1] = cell0(q.y + R, P.oy, inv) >> l;
    lo[2] = cell0(q.z - R, P.oz, inv) >> l;
    hi[2] = cell0(q.z + R, P.oz, inv) >> l;
    int sp = 0;
    for (uint32_t cz = lo[2]; cz <= hi[2]; cz++)
        for (uint32_t cy = lo[1]; cy <= hi[1]; cy++)
            for (uint32_t cx = lo[0]; cx <= hi[0]; cx++) {
                int32_t m = find_cell(g, P.hash_mask, l, cx, cy, cz);
                if (m < 0) continue;
                float d2 = cell_mindist2(P, q.x, q.y, q.z, cx, cy, cz, l);
                if (d2 > b2) continue;
                if (sp < kStack) {
                    stk[sp * stride] = make_uint2((uint32_t)m, __float_as_uint(d2));
                    ++sp;
                } else {
                    NodeHdr h = g.hdr[m];
                    scan_range(g.pts, h.start, h.start + h.count, xs, xe, q, v);
                }
            }
    dfs<V, LEAF>(g, P, q, v, stk, stride, sp, xs, xe);
}

// Full search.  `need` = number of points the seed cell must hold (k, or 1
// for the nearest neighbour).  When the visitor already has a finite radius
// (a warm start) the seed phase is skipped.
template <class V, int LEAF>
__device__ inline void search(const GridView &g, const GridParams &P, const Query &q, V &v, int need, uint2 *stk,
                              int stride)
{
    const float inv = P.inv_h0;
    uint32_t xs = 0, xe = 0;
    if (!v.have()) {
        // seed: smallest cell around q (level lmin and up) holding >= need points
        uint32_t c0x = cell0(q.x, P.ox, inv), c0y = cell0(q.y, P.oy, inv), c0z = cell0(q.z, P.oz, inv);
        int32_t seed = -1;
        for (int l = P.lmin; l < kLevels; l++) {
            int32_t m = find_cell(g, P.hash_mask, l, c0x >> l, c0y >> l, c0z >> l);
            if (m >= 0 && g.hdr[m].count >= (uint32_t)need) {
                seed = m;
                break;
            }
        }
        if (seed < 0) return;   // fewer than `need` points in the cloud
        stk[0] = make_uint2((uint32_t)seed, 0u);
        dfs<V, LEAF>(g, P, q, v, stk, stride, 1, 0u, 0u);
        NodeHdr hs = g.hdr[seed];
        xs = hs.start;
        xe = hs.start + hs.count;
    }
    cover<V, LEAF>(g, P, q, v, stk, stride, xs, xe);
}

}  // namespace pcg
