// Sparse voxel pyramid over a point cloud, built on the device.
//
// The paper's neighbour queries run on a kd-tree and its downsampling on a
// uniform voxel grid (Section 3, "Core operations").  On the GPU both roles
// are played by one structure: points are binned into a 2^16-per-axis
// uniform voxel grid, sorted by the cells' Morton keys with a stable LSD
// radix sort (coalesced tile reads, per-block digit ranking in LDS), and
// every level-L cell (2^L level-0 cells per axis) becomes a contiguous run of
// the sorted array.  The non-empty cells of the levels at and above a
// density-chosen finest level form an implicit octree (nodes per level,
// children contiguous) and are also entered in an open-addressing hash keyed
// by (level, cell), so a query can start at any cell directly.
//
// Everything is sized from the point count (an upper bound); data-dependent
// counts stay on the device, so building needs no host read-back.

#include "common.h"

namespace pcg {

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kKeyBits = 3 * kBits;                      // 48
constexpr int kPasses = (kKeyBits + kRadixBits - 1) / kRadixBits;  // 6
constexpr int kLvlThreads = 256;
constexpr int kLvlItems = 4;
constexpr int kLvlTile = kLvlThreads * kLvlItems;
constexpr uint32_t kNoStart = 0xffu;

__device__ inline uint64_t lanemask_lt()
{
    uint32_t l = __lane_id();
    return (l == 0) ? 0ull : (~0ull >> (64 - l));
}

// ---------------------------------------------------------------- bbox
__global__ void k_bbox_init(uint32_t *bb)
{
    int t = threadIdx.x;
    if (t < 3) bb[t] = 0xffffffffu;       // min (ordered)
    else if (t < 6) bb[t] = 0u;          // max (ordered)
}

__global__ void __launch_bounds__(256) k_bbox(const float *__restrict__ xyz, int64_t n, uint32_t *bb)
{
    __shared__ float red[4][6];
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        for (int a = 0; a < 3; a++) {
            float v = xyz[3 * i + a];
            mn[a] = fminf(mn[a], v);
            mx[a] = fmaxf(mx[a], v);
        }
    }
    for (int off = 32; off > 0; off >>= 1)
        for (int a = 0; a < 3; a++) {
            mn[a] = fminf(mn[a], __shfl_xor(mn[a], off));
            mx[a] = fmaxf(mx[a], __shfl_xor(mx[a], off));
        }
    int w = threadIdx.x >> 6;
    if (__lane_id() == 0)
        for (int a = 0; a < 3; a++) {
            red[w][a] = mn[a];
            red[w][3 + a] = mx[a];
        }
    __syncthreads();
    // one set of atomics per block
    if (threadIdx.x < 6) {
        int a = threadIdx.x;
        float v = red[0][a];
        for (int x = 1; x < 4; x++) v = a < 3 ? fminf(v, red[x][a]) : fmaxf(v, red[x][a]);
        bool finite = a < 3 ? v < INFINITY : v > -INFINITY;
        if (finite) {
            if (a < 3) atomicMin(&bb[a], f2ord(v));
            else atomicMax(&bb[a], f2ord(v));
        }
    }
}

__global__ void k_params(uint32_t *bb, GridParams *P, int64_t n)
{
    float lo[3], hi[3];
    float ext = 0.f, mag = 0.f;
    for (int a = 0; a < 3; a++) {
        lo[a] = ord2f(bb[a]);
        hi[a] = ord2f(bb[3 + a]);
        if (n == 0) lo[a] = hi[a] = 0.f;
        ext = fmaxf(ext, hi[a] - lo[a]);
        mag = fmaxf(mag, fmaxf(fabsf(lo[a]), fabsf(hi[a])));
    }
    if (!(ext > 0.f)) ext = 1.0f;
    // cube side: a little larger than the extent so the top face bins below 2^16
    float side = ext * (1.0f + 1.0f / 1024.0f) + mag * 1e-6f + 1e-30f;
    P->ox = lo[0];
    P->oy = lo[1];
    P->oz = lo[2];
    P->inv_h0 = (float)(1u << kBits) / side;
    P->h0 = side / (float)(1u << kBits);
    P->margin = (mag + side) * (1.0f / (1 << 20));
    P->n = (int32_t)n;
    for (int l = 0; l < kLevels; l++) {
        P->level_count[l] = 0;
        P->level_off[l] = 0;
    }
}

// ---------------------------------------------------------------- keys
__global__ void k_keys(const float *__restrict__ xyz, int64_t n, const GridParams *__restrict__ P,
                       uint64_t *__restrict__ keys)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    float ox = P->ox, oy = P->oy, oz = P->oz, inv = P->inv_h0;
    uint32_t cx = cell0(xyz[3 * i + 0], ox, inv);
    uint32_t cy = cell0(xyz[3 * i + 1], oy, inv);
    uint32_t cz = cell0(xyz[3 * i + 2], oz, inv);
    keys[i] = morton3(cx, cy, cz);
}

// ---------------------------------------------------------------- radix sort
// hist[d * nblk + b] = number of keys with digit d in tile b
__global__ void __launch_bounds__(kSortThreads) k_radix_hist(const uint64_t *__restrict__ keys, int64_t n,
                                                             int shift, uint32_t *__restrict__ hist)
{
    __shared__ uint32_t cnt[kRadix];
    int t = threadIdx.x;
    cnt[t] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortItems; r++) {
        int64_t e = base + r * kSortThreads + t;
        if (e < n) atomicAdd(&cnt[(keys[e] >> shift) & (kRadix - 1)], 1u);
    }
    __syncthreads();
    hist[(int64_t)t * gridDim.x + blockIdx.x] = cnt[t];
}

// Per-digit exclusive scan over tiles (one wave per digit, 64 tiles per
// step): hist[d * nblk + b] becomes the offset of tile b within digit d;
// tot[d] receives the digit's total.
__global__ void __launch_bounds__(256) k_radix_colscan(uint32_t *__restrict__ hist, int nblk,
                                                     uint32_t *__restrict__ tot)
{
    const int d = blockIdx.x * 4 + (threadIdx.x >> 6), lane = __lane_id();
    uint32_t carry = 0;
    for (int b0 = 0; b0 < nblk; b0 += 64) {
        int b = b0 + lane;
        uint32_t v = (b < nblk) ? hist[(int64_t)d * nblk + b] : 0u;
        uint32_t x = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            uint32_t y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (b < nblk) hist[(int64_t)d * nblk + b] = carry + x - v;
        carry += __shfl(x, 63);
    }
    if (lane == 0) tot[d] = carry;
}

// Stable scatter of one radix pass.  Each block walks its tile in rounds of
// 256 consecutive keys; the rank of a key among equal digits is its lane rank
// inside the wave (from eight ballots) plus the counts of earlier waves and
// earlier rounds, so the original order of equal digits is kept.
__global__ void __launch_bounds__(kSortThreads) k_radix_scatter(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ iin, int64_t n, int shift,
    const uint32_t *__restrict__ hist, const uint32_t *__restrict__ tot, uint64_t *__restrict__ kout,
    uint32_t *__restrict__ iout)
{
    constexpr int W = kSortThreads / 64;
    __shared__ uint32_t running[kRadix];
    __shared__ uint32_t wcnt[W][kRadix];
    __shared__ uint32_t wsum[W];
    int t = threadIdx.x, w = t >> 6;
    // digit base = exclusive scan of the digit totals (256 values, in LDS)
    {
        uint32_t v = tot[t], x = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            uint32_t y = __shfl_up(x, off);
            if (__lane_id() >= off) x += y;
        }
        if (__lane_id() == 63) wsum[w] = x;
        __syncthreads();
        uint32_t before = 0;
        for (int x2 = 0; x2 < w; x2++) before += wsum[x2];
        running[t] = before + x - v + hist[(int64_t)t * gridDim.x + blockIdx.x];
    }
    for (int x = 0; x < W; x++) wcnt[x][t] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kSortTile;
    uint64_t lt = lanemask_lt();
    for (int r = 0; r < kSortItems; r++) {
        int64_t e = base + r * kSortThreads + t;
        bool valid = e < n;
        uint64_t key = valid ? kin[e] : 0ull;
        uint32_t id = valid ? (iin ? iin[e] : (uint32_t)e) : 0u;
        uint32_t d = (uint32_t)(key >> shift) & (kRadix - 1);
        uint64_t m = __ballot(valid);
        for (int b = 0; b < kRadixBits; b++) {
            uint64_t bb = __ballot((d >> b) & 1u);
            m &= ((d >> b) & 1u) ? bb : ~bb;
        }
        uint32_t wrank = __popcll(m & lt);
        if (valid && wrank == 0) wcnt[w][d] = __popcll(m);
        __syncthreads();
        if (valid) {
            uint32_t pos = running[d] + wrank;
            for (int x = 0; x < w; x++) pos += wcnt[x][d];
            kout[pos] = key;
            iout[pos] = id;
        }
        __syncthreads();
        uint32_t tot = 0;
        for (int x = 0; x < W; x++) {
            tot += wcnt[x][t];
            wcnt[x][t] = 0;
        }
        running[t] += tot;
        __syncthreads();
    }
}

__global__ void k_gather_pts(const float *__restrict__ xyz, const uint32_t *__restrict__ idx, int64_t n,
                             float4 *__restrict__ pts)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t j = idx[i];
    pts[i] = make_float4(xyz[3 * (int64_t)j], xyz[3 * (int64_t)j + 1], xyz[3 * (int64_t)j + 2],
                         __uint_as_float(j));
}

__global__ void k_gather3(const float *__restrict__ src, const uint32_t *__restrict__ idx, int64_t n,
                          float4 *__restrict__ dst)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t j = idx[i];
    dst[i] = make_float4(src[3 * (int64_t)j], src[3 * (int64_t)j + 1], src[3 * (int64_t)j + 2], 0.f);
}

// ---------------------------------------------------------------- levels
// slev[i] = highest level at which sorted point i opens a new cell
// (kNoStart if it opens none); P->level_count[s] counts points with slev == s
__global__ void k_slev(const uint64_t *__restrict__ keys, int64_t n, uint32_t *__restrict__ slev,
                       GridParams *P)
{
    __shared__ uint32_t h[kLevels];
    int t = threadIdx.x;
    if (t < kLevels) h[t] = 0;
    __syncthreads();
    int64_t i = blockIdx.x * (int64_t)blockDim.x + t;
    if (i < n) {
        uint32_t s;
        if (i == 0) {
            s = kLevels - 1;
        } else {
            uint64_t x = keys[i] ^ keys[i - 1];
            s = x ? (uint32_t)((63 - __clzll(x)) / 3) : kNoStart;
        }
        slev[i] = s;
        if (s != kNoStart) atomicAdd(&h[s], 1u);
    }
    __syncthreads();
    if (t < kLevels && h[t]) atomicAdd(&P->level_count[t], (int)h[t]);
}

// turns the slev histogram into node counts per level, picks the finest
// level such that the pyramid from there up has at most n nodes (so leaves
// are as small as a node budget of one per point allows, also where the
// density is far above the mean), lays out the node arrays and the hash size
__global__ void k_levels(GridParams *P, int64_t n, uint32_t hash_cap_max)
{
    int32_t cnt[kLevels];
    int32_t run = 0;
    for (int l = kLevels - 1; l >= 0; l--) {
        run += P->level_count[l];
        cnt[l] = run;           // points opening a cell at level >= l = cells at level l
    }
    int lmin = kLevels - 1;
    int64_t cum = 0;
    for (int l = kLevels - 1; l >= 0; l--) {
        cum += cnt[l];
        if (cum > (n > 1 ? n : 1)) break;
        lmin = l;
    }
    int32_t off = 0;
    for (int l = 0; l < kLevels; l++) {
        P->level_count[l] = (l >= lmin) ? cnt[l] : 0;
        P->level_off[l] = off;
        if (l >= lmin) off += cnt[l];
    }
    P->lmin = lmin;
    P->n_nodes = off;
    uint32_t cap = 1024;
    while (cap < 2u * (uint32_t)off && cap < hash_cap_max) cap <<= 1;
    P->hash_mask = cap - 1;
}

// per tile of kLvlTile sorted points: number of cells each level opens
__global__ void __launch_bounds__(kLvlThreads) k_level_count(const uint32_t *__restrict__ slev, int64_t n,
                                                           const GridParams *__restrict__ P,
                                                           int32_t *__restrict__ lb)
{
    __shared__ int32_t c[kLevels];
    int t = threadIdx.x;
    if (t < kLevels) c[t] = 0;
    __syncthreads();
    int lmin = P->lmin;
    int64_t base = (int64_t)blockIdx.x * kLvlTile;
    for (int r = 0; r < kLvlItems; r++) {
        int64_t i = base + r * kLvlThreads + t;
        uint32_t s = (i < n) ? slev[i] : kNoStart;
#pragma unroll
        for (int l = 0; l < kLevels; l++) {
            if (l < lmin) continue;
            uint64_t b = __ballot(s != kNoStart && (int)s >= l);
            if (__lane_id() == 0 && b) atomicAdd(&c[l], __popcll(b));
        }
    }
    __syncthreads();
    if (t < kLevels) lb[(int64_t)blockIdx.x * kLevels + t] = c[t];
}

// exclusive scan over tiles, one wave per level
__global__ void __launch_bounds__(1024) k_level_scan(int32_t *__restrict__ lb, int nblk)
{
    int w = threadIdx.x >> 6, lane = __lane_id();
    for (int l = w; l < kLevels; l += 16) {
        int32_t carry = 0;
        for (int b0 = 0; b0 < nblk; b0 += 64) {
            int b = b0 + lane;
            int32_t v = (b < nblk) ? lb[(int64_t)b * kLevels + l] : 0;
            int32_t x = v;
            for (int off = 1; off < 64; off <<= 1) {
                int32_t y = __shfl_up(x, off);
                if (lane >= off) x += y;
            }
            if (b < nblk) lb[(int64_t)b * kLevels + l] = carry + x - v;
            carry += __shfl(x, 63);
        }
    }
}

// writes node starts, levels and first children
__global__ void __launch_bounds__(kLvlThreads) k_level_scatter(const uint32_t *__restrict__ slev, int64_t n,
                                                             const GridParams *__restrict__ P,
                                                             const int32_t *__restrict__ lb,
                                                             Node *__restrict__ nodes)
{
    constexpr int W = kLvlThreads / 64;
    __shared__ int32_t running[kLevels];
    __shared__ int32_t wtot[kLevels][W];
    int t = threadIdx.x, w = t >> 6;
    int lmin = P->lmin;
    if (t < kLevels) running[t] = lb[(int64_t)blockIdx.x * kLevels + t];
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kLvlTile;
    uint64_t lt = lanemask_lt();
    for (int r = 0; r < kLvlItems; r++) {
        int64_t i = base + r * kLvlThreads + t;
        uint32_t s = (i < n) ? slev[i] : kNoStart;
        int32_t rank[kLevels];
#pragma unroll
        for (int l = 0; l < kLevels; l++) {
            bool f = l >= lmin && s != kNoStart && (int)s >= l;
            uint64_t b = __ballot(f);
            rank[l] = __popcll(b & lt);
            if (__lane_id() == 0 && l >= lmin) wtot[l][w] = __popcll(b);
        }
        __syncthreads();
        int32_t prev = -1;
#pragma unroll
        for (int l = 0; l < kLevels; l++) {
            bool f = l >= lmin && s != kNoStart && (int)s >= l;
            int32_t pos = running[l] + rank[l];
            for (int x = 0; x < w; x++) pos += wtot[l][x];
            int32_t node = P->level_off[l] + pos;
            if (f) {
                NodeHdr h;
                h.start = (uint32_t)i;
                h.count = 0;
                h.first_child = (l > lmin) ? (uint32_t)prev : 0xffffffffu;
                h.meta = (uint32_t)l << 8;
                nodes[node].h = h;
            }
            prev = node;
        }
        __syncthreads();
        if (t < kLevels && t >= lmin) {
            int32_t s2 = 0;
            for (int x = 0; x < W; x++) s2 += wtot[t][x];
            running[t] += s2;
        }
        __syncthreads();
    }
}

__global__ void k_hash_clear(const GridParams *__restrict__ P, HSlot *__restrict__ hs)
{
    uint32_t cap = P->hash_mask + 1;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += gridDim.x * blockDim.x)
        hs[i].key = kEmptyKey;
}

// node counts, child counts, hash insertion
__global__ void k_nodes_finish(const GridParams *__restrict__ P, const uint64_t *__restrict__ keys,
                               Node *__restrict__ nodes, HSlot *__restrict__ hs)
{
    int32_t total = P->n_nodes, n = P->n, lmin = P->lmin;
    uint32_t mask = P->hash_mask;
    for (int32_t m = blockIdx.x * blockDim.x + threadIdx.x; m < total; m += gridDim.x * blockDim.x) {
        // start, first_child and the level were written by the scatter pass
        // and are only read here; each thread writes its own node's counts
        uint32_t start = nodes[m].h.start;
        uint32_t meta = nodes[m].h.meta;
        int l = (int)(meta >> 8);
        int32_t lend = P->level_off[l] + P->level_count[l];
        uint32_t next_start = (m + 1 < lend) ? nodes[m + 1].h.start : (uint32_t)n;
        nodes[m].h.count = next_start - start;
        if (l > lmin) {
            uint32_t fc = nodes[m].h.first_child;
            uint32_t next_fc = (m + 1 < lend) ? nodes[m + 1].h.first_child
                                              : (uint32_t)(P->level_off[l - 1] + P->level_count[l - 1]);
            nodes[m].h.meta = meta | (next_fc - fc);
        }
        uint64_t key = hash_key(l, keys[start] >> (3 * l));
        uint32_t s = hash_slot(key, mask);
        for (uint32_t it = 0; it <= mask; it++) {
            unsigned long long prev = atomicCAS((unsigned long long *)&hs[s].key, (unsigned long long)kEmptyKey,
                                                (unsigned long long)key);
            if (prev == kEmptyKey) {
                hs[s].val = (uint32_t)m;
                break;
            }
            s = (s + 1) & mask;
        }
    }
}

// tight boxes of the level-l nodes in level-0 cells: from their points'
// cells at the finest level, from their children's boxes above it
__global__ void k_node_boxes(const GridParams *__restrict__ P, int l, const uint64_t *__restrict__ keys,
                             Node *__restrict__ nodes)
{
    int lmin = P->lmin;
    if (l < lmin) return;
    int32_t off = P->level_off[l], end = off + P->level_count[l];
    for (int32_t m = off + blockIdx.x * blockDim.x + threadIdx.x; m < end; m += gridDim.x * blockDim.x) {
        NodeHdr h = nodes[m].h;
        uint32_t lx = 0xffffu, ly = 0xffffu, lz = 0xffffu, hx = 0, hy = 0, hz = 0;
        if (l == lmin) {
            for (uint32_t j = h.start; j < h.start + h.count; j++) {
                uint64_t k = keys[j];
                uint32_t x = compact3(k), y = compact3(k >> 1), z = compact3(k >> 2);
                lx = min(lx, x); ly = min(ly, y); lz = min(lz, z);
                hx = max(hx, x); hy = max(hy, y); hz = max(hz, z);
            }
        } else {
            uint32_t nc = node_nchild(h);
            for (uint32_t c = 0; c < nc; c++) {
                const Node &ch = nodes[h.first_child + c];
                lx = min(lx, ch.bx & 0xffffu); ly = min(ly, ch.bx >> 16); lz = min(lz, ch.by & 0xffffu);
                hx = max(hx, ch.by >> 16); hy = max(hy, ch.bz & 0xffffu); hz = max(hz, ch.bz >> 16);
            }
        }
        nodes[m].bx = lx | (ly << 16);
        nodes[m].by = lz | (hx << 16);
        nodes[m].bz = hy | (hz << 16);
        nodes[m].pad = 0;
    }
}

inline int blocks_for(int64_t n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

int64_t max_pyramid_nodes(int64_t n)
{
    // the kept levels hold at most max(n, 1) nodes in total
    return (n > 1 ? n : 1) + 1;
}

static uint32_t hash_cap_for(int64_t nodes)
{
    uint64_t cap = 1024;
    while (cap < 2ull * (uint64_t)nodes && cap < (1ull << 31)) cap <<= 1;
    return (uint32_t)cap;
}

void grid_carve(Carver &c, int64_t n, GridStore &g)
{
    int64_t nn = n > 0 ? n : 1;
    g.n = n;
    g.nblk_sort = (int)((nn + kSortTile - 1) / kSortTile);
    g.nblk_lvl = (int)((nn + kLvlTile - 1) / kLvlTile);
    g.max_nodes = max_pyramid_nodes(nn);
    g.hash_cap_max = hash_cap_for(g.max_nodes);
    g.params = c.take<GridParams>(1);
    g.bbox = c.take<uint32_t>(8);
    g.keys = c.take<uint64_t>(nn);
    g.keys_alt = c.take<uint64_t>(nn);
    g.idx = c.take<uint32_t>(nn);
    g.idx_alt = c.take<uint32_t>(nn);
    g.pts = c.take<float4>(nn);
    g.slev = c.take<uint32_t>(nn);
    g.radix_hist = c.take<uint32_t>((size_t)g.nblk_sort * kRadix);
    g.radix_tot = c.take<uint32_t>(kRadix);
    g.level_block = c.take<int32_t>((size_t)g.nblk_lvl * kLevels);
    g.node = c.take<Node>(g.max_nodes);
    g.hash = c.take<HSlot>(g.hash_cap_max);
}

size_t grid_bytes(int64_t n)
{
    Carver c(nullptr, ~(size_t)0 >> 1);
    GridStore g;
    grid_carve(c, n, g);
    return c.used();
}

hipError_t grid_build(GridStore &g, const float *xyz, hipStream_t s)
{
    const int64_t n = g.n;
    const int T = 256;
    k_bbox_init<<<1, 64, 0, s>>>(g.bbox);
    int bb_blocks = blocks_for(n, T);
    if (bb_blocks > 256) bb_blocks = 256;
    if (bb_blocks < 1) bb_blocks = 1;
    k_bbox<<<bb_blocks, T, 0, s>>>(xyz, n, g.bbox);
    k_params<<<1, 1, 0, s>>>(g.bbox, g.params, n);
    if (n > 0) {
        k_keys<<<blocks_for(n, T), T, 0, s>>>(xyz, n, g.params, g.keys);
        uint64_t *ka = g.keys, *kb = g.keys_alt;
        uint32_t *ia = nullptr, *ib = g.idx_alt;
        for (int p = 0; p < kPasses; p++) {
            int shift = p * kRadixBits;
            k_radix_hist<<<g.nblk_sort, kSortThreads, 0, s>>>(ka, n, shift, g.radix_hist);
            k_radix_colscan<<<kRadix / 4, 256, 0, s>>>(g.radix_hist, g.nblk_sort, g.radix_tot);
            k_radix_scatter<<<g.nblk_sort, kSortThreads, 0, s>>>(ka, ia, n, shift, g.radix_hist, g.radix_tot,
                                                                 kb, ib);
            // ping-pong; with an even number of passes the result lands in keys/idx
            uint64_t *tk = ka; ka = kb; kb = tk;
            if (p == 0) { ia = g.idx_alt; ib = g.idx; }
            else { uint32_t *ti = ia; ia = ib; ib = ti; }
        }
        static_assert(kPasses % 2 == 0, "sorted keys must end in the primary buffers");
        k_gather_pts<<<blocks_for(n, T), T, 0, s>>>(xyz, g.idx, n, g.pts);
        k_slev<<<blocks_for(n, T), T, 0, s>>>(g.keys, n, g.slev, g.params);
    }
    k_levels<<<1, 1, 0, s>>>(g.params, n, g.hash_cap_max);
    if (n > 0) {
        k_level_count<<<g.nblk_lvl, kLvlThreads, 0, s>>>(g.slev, n, g.params, g.level_block);
        k_level_scan<<<1, 1024, 0, s>>>(g.level_block, g.nblk_lvl);
        k_level_scatter<<<g.nblk_lvl, kLvlThreads, 0, s>>>(g.slev, n, g.params, g.level_block, g.node);
        int hb = blocks_for(g.hash_cap_max, T);
        if (hb > 4096) hb = 4096;
        k_hash_clear<<<hb, T, 0, s>>>(g.params, g.hash);
        int nb = blocks_for(g.max_nodes, T);
        if (nb > 4096) nb = 4096;
        k_nodes_finish<<<nb, T, 0, s>>>(g.params, g.keys, g.node, g.hash);
        int bxb = blocks_for(n, T);
        if (bxb > 2048) bxb = 2048;
        for (int l = 0; l < kLevels; l++) k_node_boxes<<<bxb, T, 0, s>>>(g.params, l, g.keys, g.node);
    }
    return hipGetLastError();
}

hipError_t grid_gather3(const GridStore &g, const float *src3, float4 *dst, hipStream_t s)
{
    if (g.n > 0) k_gather3<<<blocks_for(g.n, 256), 256, 0, s>>>(src3, g.idx, g.n, dst);
    return hipGetLastError();
}

}  // namespace pcg
