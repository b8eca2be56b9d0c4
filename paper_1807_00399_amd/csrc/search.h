// Exact nearest-neighbour search over the sparse voxel pyramid.
//
// One lane answers one query.  The traversal is generic over a candidate
// visitor V (the ranking and the running search radius live there):
//   bool  V::have()          a finite radius is already known (warm start)
//   float V::bound2()        current search radius^2 (float32, inclusive)
//   void  V::visit(x,y,z,j,p,m) offer sorted point j (coordinates p) of node m
//
// The search has two phases:
//   seed  - the smallest cell containing the query that holds `need` points
//           is searched first, which gives a finite radius;
//   cover - the cells of the coarsest useful level (width >= 2R) that meet
//           the ball of radius R are searched depth-first, children nearest
//           first, skipping every cell whose box is farther than the current
//           radius and every point range the seed already contributed.
// A node is skipped by its tight float32 box, whose distance never exceeds
// the key of a point inside it; a grid cell (cover phase) by its box shrunk
// by an absolute margin and a relative factor.  So nothing is skipped unless
// every point in it is strictly outside the radius: no candidate inside the
// radius is ever missed, ties included.
//
// The traversal is bound by memory latency, so independent loads are issued
// together: the up-to-8 children of a node, the up-to-8 cells of the cover
// and groups of seed levels each cost one round trip, not one per item.
#pragma once

#include "common.h"

namespace pcg {

constexpr int kStack = 32;              // default per-lane DFS stack entries
constexpr int kStackNear = 24;          // nearest-neighbour searches of ICP: shallower stacks, higher occupancy
// Whether stack entries carry their push-time distance (below).  Off for
// both searches: a pop beyond the bound then still loads its node, but the
// 8-byte entries double the stack's LDS, and the waves lost to that cost
// more than the loads saved (ICP loops 20-30 % slower, k-NN and normals
// 15-30 % slower).
constexpr bool kSearchDist = false;     // k-NN and normals
constexpr bool kNearDist = false;       // ICP correspondences
constexpr int kVisitBudget = 1 << 20;   // node pops per DFS; only a corrupted tree reaches it

// One lane's DFS stack in LDS: a column of CAP entries `stride` apart (the
// lanes of a block interleave, so a wave's accesses are conflict-free).
// With DIST, an entry also holds a lower bound of the squared distance from
// the query to the node's points, taken when it was pushed (the node's box
// distance for a child, the cell's for a cover cell), so a pop whose node
// lies beyond the bound tightened since is dropped without loading the node.
template <int CAP, bool DIST>
struct Stack;

template <int CAP>
struct Stack<CAP, false> {
    static constexpr int cap = CAP;
    static constexpr int words = CAP;   // 4-byte LDS words per lane
    uint32_t *p;
    int stride;
    __device__ void put(int sp, uint32_t id, float) const { p[sp * stride] = id; }
    __device__ uint32_t get(int sp, float &d) const
    {
        d = 0.f;
        return p[sp * stride];
    }
};

template <int CAP>
struct Stack<CAP, true> {
    static constexpr int cap = CAP;
    static constexpr int words = 2 * CAP;
    uint2 *p;
    int stride;
    __device__ void put(int sp, uint32_t id, float d) const { p[sp * stride] = make_uint2(id, __float_as_uint(d)); }
    __device__ uint32_t get(int sp, float &d) const
    {
        const uint2 e = p[sp * stride];
        d = __uint_as_float(e.y);
        return e.x;
    }
};

// the stacks of the k-NN / normals searches and of the ICP correspondence
// search; `base` is the block's LDS array (S::words * threads words, 8-byte
// aligned), lane t's column starts at entry t
template <class S>
__device__ inline S lane_stack(uint32_t *base, int threads)
{
    if constexpr (S::words == S::cap) return S{base + threadIdx.x, threads};
    else return S{reinterpret_cast<uint2 *>(base) + threadIdx.x, threads};
}
using SearchStack = Stack<kStack, kSearchDist>;
using NearStack = Stack<kStackNear, kNearDist>;

__device__ inline uint64_t enc_cand(float key, float w) { return ((uint64_t)__float_as_uint(key) << 32) | __float_as_uint(w); }

// k best candidates by (float32 key, original index): the k-NN definition;
// with a finite cap2, only candidates with key <= cap2 (hybrid
// neighbourhoods: the k nearest within a radius).
template <int KT>
struct TopK {
    uint64_t h[KT];     // ascending; ~0 = empty; 0 = padding when k < KT
    float cap2;         // inclusive key limit, +inf for plain k-NN

    __device__ void init(int k, float cap = INFINITY)
    {
#pragma unroll
        for (int s = 0; s < KT; s++) h[s] = (s < KT - k) ? 0ull : ~0ull;
        cap2 = cap;
    }
    __device__ bool have() const { return h[KT - 1] != ~0ull; }
    __device__ float bound2() const
    {
        return have() ? fminf(__uint_as_float((uint32_t)(h[KT - 1] >> 32)), cap2) : cap2;
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
    __device__ void visit(float qx, float qy, float qz, uint32_t, const float4 &p, uint32_t)
    {
        float key = knn_key(p.x, p.y, p.z, qx, qy, qz);
        if (key <= cap2) insert(enc_cand(key, p.w));
    }
};

// Every candidate with key <= r2 (radius neighbourhoods): count, sums of
// the offsets d = p - q and of their products, in float64 (offsets of
// float32 values are exact in float64).
struct RadiusCov {
    float r2;
    int32_t m;
    double sx, sy, sz, sxx, sxy, sxz, syy, syz, szz;

    __device__ void init(float radius2)
    {
        r2 = radius2;
        m = 0;
        sx = sy = sz = sxx = sxy = sxz = syy = syz = szz = 0.0;
    }
    __device__ bool have() const { return true; }
    __device__ float bound2() const { return r2; }
    __device__ void visit(float qx, float qy, float qz, uint32_t, const float4 &p, uint32_t)
    {
        if (knn_key(p.x, p.y, p.z, qx, qy, qz) <= r2) {
            double dx = (double)p.x - (double)qx, dy = (double)p.y - (double)qy, dz = (double)p.z - (double)qz;
            m++;
            sx += dx; sy += dy; sz += dz;
            sxx += dx * dx; sxy += dx * dy; sxz += dx * dz;
            syy += dy * dy; syz += dy * dz; szz += dz * dz;
        }
    }
};

struct Query {
    float x, y, z;
};

// scan sorted points [s, e) of node m minus the excluded run [xs, xe)
template <class V>
__device__ inline void scan_range(const float4 *__restrict__ pts, uint32_t s, uint32_t e, uint32_t xs,
                                  uint32_t xe, const Query &q, V &v, uint32_t m)
{
    uint32_t a0 = s, a1 = e, b0 = e, b1 = e;
    if (xs < xe && xs < e && xe > s) {   // overlap with the excluded run (nested or disjoint)
        a1 = xs > s ? xs : s;
        b0 = xe < e ? xe : e;
    }
    // four independent loads per round trip
    for (uint32_t j = a0; j < a1; j += 4) {
        float4 p[4];
#pragma unroll
        for (int u = 0; u < 4; u++)
            if (j + u < a1) p[u] = pts[j + u];
#pragma unroll
        for (int u = 0; u < 4; u++)
            if (j + u < a1) v.visit(q.x, q.y, q.z, j + u, p[u], m);
    }
    for (uint32_t j = b0; j < b1; j += 4) {
        float4 p[4];
#pragma unroll
        for (int u = 0; u < 4; u++)
            if (j + u < b1) p[u] = pts[j + u];
#pragma unroll
        for (int u = 0; u < 4; u++)
            if (j + u < b1) v.visit(q.x, q.y, q.z, j + u, p[u], m);
    }
}

// continue a linear probe of `key` from slot s of cloud P's hash region
// (the first slot held another key)
__device__ inline int32_t probe_from(const GridView &g, const GridParams &P, uint64_t key, uint32_t s)
{
    const HSlot *hs = g.hash + P.hash_base;
    for (uint32_t it = 1; it < P.hash_cap; it++) {
        s = next_slot(s, P.hash_cap);
        HSlot e = hs[s];
        if (e.key == key) return (int32_t)e.val;
        if (e.key == kEmptyKey) return -1;
    }
    return -1;
}

// ascending sort of 8 words: Batcher's odd-even merge network
__device__ inline void cmp_swap(uint32_t *k, int i, int j)
{
    const uint32_t a = k[i], b = k[j];
    k[i] = a < b ? a : b;
    k[j] = a < b ? b : a;
}
__device__ inline void sort8u(uint32_t *k)
{
    cmp_swap(k, 0, 1); cmp_swap(k, 2, 3); cmp_swap(k, 4, 5); cmp_swap(k, 6, 7);
    cmp_swap(k, 0, 2); cmp_swap(k, 1, 3); cmp_swap(k, 4, 6); cmp_swap(k, 5, 7);
    cmp_swap(k, 1, 2); cmp_swap(k, 5, 6);
    cmp_swap(k, 0, 4); cmp_swap(k, 1, 5); cmp_swap(k, 2, 6); cmp_swap(k, 3, 7);
    cmp_swap(k, 2, 4); cmp_swap(k, 3, 5);
    cmp_swap(k, 1, 2); cmp_swap(k, 3, 4); cmp_swap(k, 5, 6);
}

// Depth-first search from the nodes already on the stack (sp entries); a
// node whose children would overflow the stack is scanned as a leaf.
template <class V, int LEAF, class S>
__device__ inline void dfs(const GridView &g, const GridParams &P, const Query &q, V &v, const S &stk, int sp,
                           uint32_t xs, uint32_t xe)
{
    for (int visits = 0; sp > 0 && visits < kVisitBudget; visits++) {
        --sp;
        float dpush;
        uint32_t m = stk.get(sp, dpush);
        float b2 = v.bound2();
        if (dpush > b2) continue;   // beyond the bound: the node is not loaded
        Node nd = g.node[m];
        const NodeHdr &h = nd.h;
        if (node_mindist2(nd, q.x, q.y, q.z) > b2) continue;
        if (h.start >= xs && h.start + h.count <= xe) continue;      // already searched
        uint32_t nc = node_nchild(h);
        bool leaf = (h.count <= (uint32_t)LEAF) || node_level(h) == P.lmin || sp + (int)nc > S::cap;
        if (leaf) {
            scan_range(g.pts, h.start, h.start + h.count, xs, xe, q, v, m);
            continue;
        }
        // all children boxes in one round trip
        const uint32_t fc = h.first_child;
        float d[8];
#pragma unroll
        for (int c = 0; c < 8; c++) {
            // padding slots are never pushed, even when the bound is still
            // infinite
            d[c] = c < (int)nc ? node_box_mindist2(g.node, fc + c, q.x, q.y, q.z) : NAN;
        }
        // nearest child last (searched next), the others in index order
        // (cheaper than sorting all eight, and as fast to tighten the bound)
        int best = 0;
        float bd = d[0];
#pragma unroll
        for (int c = 1; c < 8; c++) {
            bool lt = d[c] < bd;
            bd = lt ? d[c] : bd;
            best = lt ? c : best;
        }
#pragma unroll
        for (int c = 0; c < 8; c++) {
            if (c != best && d[c] <= b2) {   // false for padding (NaN)
                stk.put(sp, fc + c, d[c]);
                ++sp;
            }
        }
        if (bd <= b2) {
            stk.put(sp, fc + best, bd);
            ++sp;
        }
    }
}

// level whose cells are at least 2R wide for the radius of b2 (17 when b2 is
// not finite)
__device__ inline int cover_level(const GridParams &P, float b2)
{
    if (!(b2 < INFINITY)) return kLevels;
    float R = sqrtf(b2) * (1.0f + 1.0f / (1 << 20)) + P.margin;
    // smallest l >= lmin with h0 * 2^l * (1 - 1/1024) >= 2R: the exponent of
    // the (slightly enlarged) ratio, rounded up
    float ratio = 2.0f * R / (P.h0 * (1.0f - 1.0f / 1024)) * (1.0f + 1.0f / (1 << 20));
    uint32_t b = __float_as_uint(ratio);
    int e = (int)(b >> 23) - 127 + ((b & 0x7fffffu) != 0u);
    int l = e > P.lmin ? e : P.lmin;
    return l < kLevels - 1 ? l : kLevels - 1;
}

// Cover phase: every cell meeting the ball of the visitor's current radius,
// nearest cell searched first.  Which of the (at most 8) cells meet the ball
// is decided from their boxes before any memory access; their hash probes
// go out four at a time, which keeps the live registers (and so the
// occupancy of the kernels that search) lower than eight probes in flight.
template <class V, int LEAF, class S>
__device__ inline void cover(const GridView &g, const GridParams &P, const Query &q, V &v, const S &stk, uint32_t xs,
                             uint32_t xe)
{
    const float inv = P.inv_h0;
    float b2 = v.bound2();
    if (!(b2 < INFINITY)) return;
    float R = sqrtf(b2) * (1.0f + 1.0f / (1 << 20)) + P.margin;
    // coarsest needed level: cell width >= 2R (with slack) so the ball box
    // meets at most two cells per axis
    int l = cover_level(P, b2);
    uint32_t lx = cell0(q.x - R, P.ox, inv) >> l, hx = cell0(q.x + R, P.ox, inv) >> l;
    uint32_t ly = cell0(q.y - R, P.oy, inv) >> l, hy = cell0(q.y + R, P.oy, inv) >> l;
    uint32_t lz = cell0(q.z - R, P.oz, inv) >> l, hz = cell0(q.z + R, P.oz, inv) >> l;
    int sp = 0;
    const HSlot *hs = g.hash + P.hash_base;
    if (hx - lx <= 1 && hy - ly <= 1 && hz - lz <= 1) {
        // up to 8 cells (bit 0: x + 1, bit 1: y + 1, bit 2: z + 1); only
        // those meeting the ball are probed.  Sort words: the cell's
        // distance bits with the cell number in the low 3 bits (distances
        // are non-negative, so their bits order as integers; the 3 bits
        // dropped only reorder near-ties), cells outside the ball last.
        uint32_t sk[8];
#pragma unroll
        for (int c = 0; c < 8; c++) {
            uint32_t cx = lx + (c & 1), cy = ly + ((c >> 1) & 1), cz = lz + (c >> 2);
            bool ok = cx <= hx && cy <= hy && cz <= hz;
            float dc = ok ? cell_mindist2(P, q.x, q.y, q.z, cx, cy, cz, l) : INFINITY;
            sk[c] = dc <= b2 ? ((__float_as_uint(dc) & ~7u) | (uint32_t)c) : 0xffffffffu;
        }
        sort8u(sk);
        // keys of the upper neighbours derived from the lower corner's key
        const uint64_t m0 = morton3(lx, ly, lz);
        const uint64_t mx = hx > lx ? morton_inc<0>(m0) : m0;
        const uint64_t ymask = 0x249249249249ull << 1;
        const uint64_t yd = hy > ly ? morton_inc<1>(m0) & ymask : m0 & ymask;
        const uint64_t zmask = 0x249249249249ull << 2;
        const uint64_t zd = hz > lz ? morton_inc<2>(m0) & zmask : m0 & zmask;
        // hash probes four at a time: the farther four first (a round only
        // when one of them meets the ball), pushed before the nearer four so
        // the nearest cell is searched first
#pragma unroll
        for (int h = 4; h >= 0; h -= 4) {
            if (sk[h] == 0xffffffffu) continue;   // sorted: none of the four meets the ball
            uint64_t key[4];
            uint32_t slot[4];
            uint64_t hk[4];
            int32_t node[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const uint32_t c = sk[h + u] & 7u;
                const bool in = sk[h + u] != 0xffffffffu;
                const uint64_t xm = (c & 1) ? mx : m0;
                const uint64_t mk = (xm & ~(ymask | zmask)) | (((c >> 1) & 1) ? yd : (m0 & ymask)) |
                                    ((c >> 2) ? zd : (m0 & zmask));
                key[u] = hash_key(l, mk);
                slot[u] = hash_slot(key[u], P.hash_cap);
                HSlot e = in ? hs[slot[u]] : HSlot{kEmptyKey, 0u, 0u};
                hk[u] = e.key;
                node[u] = (e.key == key[u]) ? (int32_t)e.val : -1;
            }
#pragma unroll
            for (int u = 0; u < 4; u++)
                if (sk[h + u] != 0xffffffffu && hk[u] != key[u] && hk[u] != kEmptyKey)
                    node[u] = probe_from(g, P, key[u], slot[u]);
#pragma unroll
            for (int u = 3; u >= 0; u--) {
                if (node[u] >= 0) {
                    stk.put(sp, (uint32_t)node[u], __uint_as_float(sk[h + u] & ~7u));
                    ++sp;
                }
            }
        }
    } else {
        // rounding made the ball box span three cells on some axis
        for (uint32_t cz = lz; cz <= hz; cz++)
            for (uint32_t cy = ly; cy <= hy; cy++)
                for (uint32_t cx = lx; cx <= hx; cx++) {
                    int32_t m = find_cell(g, P, l, cx, cy, cz);
                    float dc = cell_mindist2(P, q.x, q.y, q.z, cx, cy, cz, l);
                    if (m < 0 || dc > b2) continue;
                    if (sp < S::cap) {
                        stk.put(sp, (uint32_t)m, dc);
                        ++sp;
                    } else {
                        NodeHdr h = g.node[m].h;
                        scan_range(g.pts, h.start, h.start + h.count, xs, xe, q, v, (uint32_t)m);
                    }
                }
    }
    dfs<V, LEAF>(g, P, q, v, stk, sp, xs, xe);
}

// smallest cell (level lmin and up) around q holding >= need points, or -1;
// levels are probed four at a time
__device__ inline int32_t seed_cell(const GridView &g, const GridParams &P, const Query &q, int need)
{
    const float inv = P.inv_h0;
    uint32_t c0x = cell0(q.x, P.ox, inv), c0y = cell0(q.y, P.oy, inv), c0z = cell0(q.z, P.oz, inv);
    // the level-l cell's key is the level-0 key shifted right by 3l
    const uint64_t m0 = morton3(c0x, c0y, c0z);
    const HSlot *hs = g.hash + P.hash_base;
    for (int l0 = P.lmin; l0 < kLevels; l0 += 4) {
        uint64_t key[4];
        uint32_t slot[4];
        uint64_t hk[4];
        int32_t node[4];
#pragma unroll
        for (int t = 0; t < 4; t++) {
            int l = l0 + t;
            bool ok = l < kLevels;
            int ls = ok ? l : 0;
            key[t] = hash_key(ls, m0 >> (3 * ls));
            slot[t] = hash_slot(key[t], P.hash_cap);
            HSlot e = ok ? hs[slot[t]] : HSlot{kEmptyKey, 0u, 0u};
            hk[t] = e.key;
            node[t] = (e.key == key[t]) ? (int32_t)e.val : -1;
        }
#pragma unroll
        for (int t = 0; t < 4; t++)
            if (hk[t] != key[t] && hk[t] != kEmptyKey) node[t] = probe_from(g, P, key[t], slot[t]);
        uint32_t cnt[4];
#pragma unroll
        for (int t = 0; t < 4; t++) cnt[t] = node[t] >= 0 ? g.node[node[t]].h.count : 0u;
#pragma unroll
        for (int t = 0; t < 4; t++)
            if (cnt[t] >= (uint32_t)need) return node[t];
    }
    return -1;
}

// Warm start: when the ball of the visitor's radius around q lies inside the
// cell of node m (record nd, a node holding the previous answer, whose point
// p0 fixes the cell), every candidate is in m, so scanning m alone is exact.  Returns
// false (nothing scanned) when the ball leaves the cell.
template <class V>
__device__ inline bool search_in_node(const GridView &g, const GridParams &P, const Query &q, V &v, uint32_t m,
                                      const Node &nd, const float4 &p0)
{
    float b2 = v.bound2();
    if (!(b2 < INFINITY)) return false;
    int l = node_level(nd.h);
    const float inv = P.inv_h0;
    float R = sqrtf(b2) * (1.0f + 1.0f / (1 << 20)) + P.margin;
    uint32_t cx = cell0(p0.x, P.ox, inv) >> l, cy = cell0(p0.y, P.oy, inv) >> l, cz = cell0(p0.z, P.oz, inv) >> l;
    bool inside = (cell0(q.x - R, P.ox, inv) >> l) == cx && (cell0(q.x + R, P.ox, inv) >> l) == cx &&
                  (cell0(q.y - R, P.oy, inv) >> l) == cy && (cell0(q.y + R, P.oy, inv) >> l) == cy &&
                  (cell0(q.z - R, P.oz, inv) >> l) == cz && (cell0(q.z + R, P.oz, inv) >> l) == cz;
    if (!inside) return false;
    scan_range(g.pts, nd.h.start, nd.h.start + nd.h.count, 0u, 0u, q, v, m);
    return true;
}

constexpr int32_t kSeedNone = -2;   // search_seed: no seed, the cap alone is covered

// First step of a search by a visitor that holds no candidate yet and whose
// radius is cap2 (`need` = number of points the seed cell must hold: k, or 1
// for the nearest neighbour): the smallest cell around q holding `need`
// points, searched first so the cover starts from a small radius; kSeedNone
// when a finite cap no larger than a few finest cells is cheap to cover
// alone; -1 when the cloud holds fewer than `need` points.  Callers with a
// large visitor (a k-NN list) take it before setting the visitor up, so the
// list's registers are not held across these hash probes.
__device__ inline int32_t search_seed(const GridView &g, const GridParams &P, const Query &q, int need, float cap2)
{
    if (cap2 < INFINITY && cover_level(P, cap2) <= P.lmin + 2) return kSeedNone;
    return seed_cell(g, P, q, need);
}

// The rest of a search from the result of search_seed: the seed cell
// depth-first, then the cover of the remaining ball without that cell.
template <class V, int LEAF, class S>
__device__ inline void search_from(const GridView &g, const GridParams &P, const Query &q, V &v, int32_t seed,
                                   const S &stk)
{
    if (seed == -1) return;   // fewer than `need` points in the cloud
    uint32_t xs = 0, xe = 0;
    if (seed >= 0) {
        stk.put(0, (uint32_t)seed, 0.f);
        dfs<V, LEAF>(g, P, q, v, stk, 1, 0u, 0u);
        NodeHdr hs = g.node[seed].h;
        xs = hs.start;
        xe = hs.start + hs.count;
    }
    cover<V, LEAF>(g, P, q, v, stk, xs, xe);
}

// Full search.  When the visitor already has a candidate (a warm start) the
// seed phase is skipped and the cover starts from its radius.
template <class V, int LEAF, class S>
__device__ inline void search(const GridView &g, const GridParams &P, const Query &q, V &v, int need, const S &stk)
{
    // one inlined cover (two copies of it grew the ICP kernel's code, and it
    // ran slower)
    const int32_t seed = v.have() ? kSeedNone : search_seed(g, P, q, need, v.bound2());
    search_from<V, LEAF>(g, P, q, v, seed, stk);
}

}  // namespace pcg
