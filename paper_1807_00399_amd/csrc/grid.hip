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
// per cloud: bbox as ordered uints (min x,y,z then max x,y,z), slev histogram
__global__ void k_cloud_init(int nc, uint32_t *__restrict__ bb, int32_t *__restrict__ clev)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nc * 6; i += gridDim.x * blockDim.x)
        bb[i] = (i % 6) < 3 ? 0xffffffffu : 0u;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nc * kLevels; i += gridDim.x * blockDim.x)
        clev[i] = 0;
}

__global__ void k_single_cloud(int64_t *off, int64_t n)
{
    off[0] = 0;
    off[1] = n;
}

// Tiles of kBoxTile points; a tile is reduced separately for each cloud it
// meets (clouds are contiguous, so usually one or two), one set of atomics
// per (tile, cloud).
constexpr int kBoxTile = 4096;

__global__ void __launch_bounds__(256) k_bbox(const float *__restrict__ xyz, const int64_t *__restrict__ off,
                                              int nc, uint32_t *bb)
{
    __shared__ float red[4][6];
    const int64_t n = off[nc];
    for (int64_t t0 = (int64_t)blockIdx.x * kBoxTile; t0 < n; t0 += (int64_t)gridDim.x * kBoxTile) {
        int64_t t1 = t0 + kBoxTile < n ? t0 + kBoxTile : n;
        int c0 = cloud_of(off, nc, t0), c1 = cloud_of(off, nc, t1 - 1);
        for (int c = c0; c <= c1; c++) {
            int64_t a = off[c] > t0 ? off[c] : t0, b = off[c + 1] < t1 ? off[c + 1] : t1;
            float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
            for (int64_t i = a + threadIdx.x; i < b; i += blockDim.x)
                for (int k = 0; k < 3; k++) {
                    float v = xyz[3 * i + k];
                    mn[k] = fminf(mn[k], v);
                    mx[k] = fmaxf(mx[k], v);
                }
            for (int o = 32; o > 0; o >>= 1)
                for (int k = 0; k < 3; k++) {
                    mn[k] = fminf(mn[k], __shfl_xor(mn[k], o));
                    mx[k] = fmaxf(mx[k], __shfl_xor(mx[k], o));
                }
            int w = threadIdx.x >> 6;
            if (__lane_id() == 0)
                for (int k = 0; k < 3; k++) {
                    red[w][k] = mn[k];
                    red[w][3 + k] = mx[k];
                }
            __syncthreads();
            if (threadIdx.x < 6) {
                int k = threadIdx.x;
                float v = red[0][k];
                for (int x = 1; x < 4; x++) v = k < 3 ? fminf(v, red[x][k]) : fmaxf(v, red[x][k]);
                bool finite = k < 3 ? v < INFINITY : v > -INFINITY;
                if (finite) {
                    if (k < 3) atomicMin(&bb[6 * c + k], f2ord(v));
                    else atomicMax(&bb[6 * c + k], f2ord(v));
                }
            }
            __syncthreads();
        }
    }
}

__global__ void k_params(const uint32_t *__restrict__ bb, const int64_t *__restrict__ off, int nc,
                         GridParams *__restrict__ P)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    int64_t n = off[c + 1] - off[c];
    float lo[3], hi[3];
    float ext = 0.f, mag = 0.f;
    for (int a = 0; a < 3; a++) {
        lo[a] = ord2f(bb[6 * c + a]);
        hi[a] = ord2f(bb[6 * c + 3 + a]);
        if (n == 0) lo[a] = hi[a] = 0.f;
        ext = fmaxf(ext, hi[a] - lo[a]);
        mag = fmaxf(mag, fmaxf(fabsf(lo[a]), fabsf(hi[a])));
    }
    if (!(ext > 0.f)) ext = 1.0f;
    // cube side: a little larger than the extent so the top face bins below 2^16
    float side = ext * (1.0f + 1.0f / 1024.0f) + mag * 1e-6f + 1e-30f;
    GridParams p;
    p.ox = lo[0];
    p.oy = lo[1];
    p.oz = lo[2];
    p.inv_h0 = (float)(1u << kBits) / side;
    p.h0 = side / (float)(1u << kBits);
    p.margin = (mag + side) * (1.0f / (1 << 20));
    p.n = (int32_t)n;
    p.base = (int32_t)off[c];
    p.lmin = kLevels - 1;
    p.n_nodes = 0;
    p.hash_base = 0;
    p.hash_cap = 0;
    P[c] = p;
}

// ---------------------------------------------------------------- keys
__global__ void k_keys(const float *__restrict__ xyz, const int64_t *__restrict__ off, int nc,
                       const GridParams *__restrict__ P, uint64_t *__restrict__ keys)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= off[nc]) return;
    int c = nc > 1 ? cloud_of(off, nc, i) : 0;
    const GridParams &p = P[c];
    uint32_t cx = cell0(xyz[3 * i + 0], p.ox, p.inv_h0);
    uint32_t cy = cell0(xyz[3 * i + 1], p.oy, p.inv_h0);
    uint32_t cz = cell0(xyz[3 * i + 2], p.oz, p.inv_h0);
    keys[i] = ((uint64_t)c << kCloudShift) | morton3(cx, cy, cz);
}

// the cloud index of every key fits above its Morton bits
static_assert(PCGPU_MAX_CLOUDS <= (1 << (64 - kCloudShift)), "cloud indices must fit above the Morton key");

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

// Exclusive scan, in place, of the n values a[0], a[stride], ... by one
// wave, 64 values per step; the loads of kAhead steps go out together (the
// running total is the only dependence between steps).  Returns the total.
template <class T>
__device__ inline T wave_excl_scan(T *a, int64_t stride, int n)
{
    constexpr int kAhead = 8;
    const int lane = __lane_id();
    T carry = 0;
    for (int b0 = 0; b0 < n; b0 += 64 * kAhead) {
        T v[kAhead];
#pragma unroll
        for (int u = 0; u < kAhead; u++) {
            const int b = b0 + 64 * u + lane;
            v[u] = b < n ? a[(int64_t)b * stride] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kAhead; u++) {
            const int b = b0 + 64 * u + lane;
            T x = v[u];
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                T y = __shfl_up(x, off);
                if (lane >= off) x += y;
            }
            if (b < n) a[(int64_t)b * stride] = carry + x - v[u];
            carry += __shfl(x, 63);
        }
    }
    return carry;
}

// Per-digit exclusive scan over tiles (one wave per digit):
// hist[d * nblk + b] becomes the offset of tile b within digit d; tot[d]
// receives the digit's total.
__global__ void __launch_bounds__(256) k_radix_colscan(uint32_t *__restrict__ hist, int nblk,
                                                     uint32_t *__restrict__ tot)
{
    const int d = blockIdx.x * 4 + (threadIdx.x >> 6);
    const uint32_t total = wave_excl_scan(hist + (int64_t)d * nblk, 1, nblk);
    if (__lane_id() == 0) tot[d] = total;
}

// exclusive prefix sum of one value per thread of a 256-thread block (all
// threads call it); ws: 4 words of LDS
__device__ inline uint32_t block_excl_scan256(uint32_t v, uint32_t *ws)
{
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(x, off);
        if (__lane_id() >= off) x += y;
    }
    const int w = threadIdx.x >> 6;
    if (__lane_id() == 63) ws[w] = x;
    __syncthreads();
    uint32_t before = 0;
    for (int x2 = 0; x2 < w; x2++) before += ws[x2];
    __syncthreads();   // ws may be reused after the call
    return before + x - v;
}

// Stable scatter of one radix pass.  A block ranks its tile of kSortTile
// keys in rounds of 256 (the rank of a key among equal digits is its lane
// rank inside the wave, from eight ballots, plus the counts of earlier waves
// and earlier rounds, so the original order of equal digits is kept), places
// them in LDS in digit order, and then writes each digit's run to its place
// in the output with consecutive lanes on consecutive addresses: the writes
// coalesce (placed straight from its round, a key landed next to about one
// other key of its digit).
__global__ void __launch_bounds__(kSortThreads) k_radix_scatter(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ iin, int64_t n, int shift,
    const uint32_t *__restrict__ hist, const uint32_t *__restrict__ tot, uint64_t *__restrict__ kout,
    uint32_t *__restrict__ iout)
{
    static_assert(kSortThreads == kRadix, "one thread per digit");
    constexpr int W = kSortThreads / 64;
    __shared__ uint64_t skey[kSortTile];
    __shared__ uint32_t sidx[kSortTile];
    __shared__ uint32_t running[kRadix];   // next tile-local position of each digit
    __shared__ int64_t delta[kRadix];      // output position minus tile-local position, per digit
    __shared__ uint16_t wcnt[W][kRadix];
    __shared__ uint32_t ws[W];
    const int t = threadIdx.x, w = t >> 6, nblk = gridDim.x, b = blockIdx.x;
    const int64_t base = (int64_t)b * kSortTile;
    {
        // digit t: this tile's count (offsets of consecutive tiles within the
        // digit differ by it), its start inside the tile, and its place in
        // the output (digit base + this tile's offset within the digit)
        const uint32_t off_b = hist[(int64_t)t * nblk + b];
        const uint32_t next = b + 1 < nblk ? hist[(int64_t)t * nblk + b + 1] : tot[t];
        const uint32_t local = block_excl_scan256(next - off_b, ws);
        const uint32_t dbase = block_excl_scan256(tot[t], ws);
        running[t] = local;
        delta[t] = (int64_t)dbase + off_b - local;
    }
    for (int x = 0; x < W; x++) wcnt[x][t] = 0;
    __syncthreads();
    const uint64_t lt = lanemask_lt();
    for (int r = 0; r < kSortItems; r++) {
        const int64_t e = base + r * kSortThreads + t;
        const bool valid = e < n;
        const uint64_t key = valid ? kin[e] : 0ull;
        const uint32_t id = valid ? (iin ? iin[e] : (uint32_t)e) : 0u;
        const uint32_t d = (uint32_t)(key >> shift) & (kRadix - 1);
        uint64_t m = __ballot(valid);
        for (int bit = 0; bit < kRadixBits; bit++) {
            const uint64_t bb = __ballot((d >> bit) & 1u);
            m &= ((d >> bit) & 1u) ? bb : ~bb;
        }
        const uint32_t wrank = __popcll(m & lt);
        if (valid && wrank == 0) wcnt[w][d] = (uint16_t)__popcll(m);
        __syncthreads();
        if (valid) {
            uint32_t pos = running[d] + wrank;
            for (int x = 0; x < w; x++) pos += wcnt[x][d];
            skey[pos] = key;
            sidx[pos] = id;
        }
        __syncthreads();
        uint32_t cnt = 0;
        for (int x = 0; x < W; x++) {
            cnt += wcnt[x][t];
            wcnt[x][t] = 0;
        }
        running[t] += cnt;
        __syncthreads();
    }
    // the tile in digit order: runs of equal digits go to consecutive
    // output positions
    const int64_t rem = n - base;
    const int tile_n = rem < kSortTile ? (int)rem : kSortTile;
    for (int x = t; x < tile_n; x += kSortThreads) {
        const uint64_t key = skey[x];
        const int64_t pos = delta[(uint32_t)(key >> shift) & (kRadix - 1)] + x;
        kout[pos] = key;
        iout[pos] = sidx[x];
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

// ---------------------------------------------------------------- levels
// slev[i] = highest level at which sorted point i opens a new cell of its
// cloud (kNoStart if it opens none; the first point of a cloud opens its
// root, level 16); clev[c * kLevels + s] counts cloud c's points with slev == s
__global__ void k_slev(const uint64_t *__restrict__ keys, int64_t n, uint32_t *__restrict__ slev,
                       int32_t *__restrict__ clev)
{
    __shared__ int32_t h[kLevels];
    int t = threadIdx.x;
    if (t < kLevels) h[t] = 0;
    __syncthreads();
    int64_t i0 = (int64_t)blockIdx.x * blockDim.x;
    int c0 = key_cloud(keys[i0 < n ? i0 : n - 1]);
    int64_t i = i0 + t;
    if (i < n) {
        uint64_t k = keys[i];
        uint32_t s;
        if (i == 0) {
            s = kLevels - 1;
        } else {
            uint64_t x = k ^ keys[i - 1];
            s = x ? (uint32_t)((63 - __clzll(x)) / 3) : kNoStart;
            if (s != kNoStart && s > (uint32_t)(kLevels - 1)) s = kLevels - 1;   // a new cloud
        }
        slev[i] = s;
        if (s != kNoStart) {
            int c = key_cloud(k);
            // the block's first cloud is counted in LDS, later ones directly
            if (c == c0) atomicAdd(&h[s], 1);
            else atomicAdd(&clev[c * kLevels + s], 1);
        }
    }
    __syncthreads();
    if (t < kLevels && h[t]) atomicAdd(&clev[c0 * kLevels + t], h[t]);
}

// Per cloud: node counts per level from the slev histogram, the finest level
// (the finest such that the levels from there up hold at most budget * n
// nodes, so leaves are as small as that node budget allows, also where the
// density is far above the mean), and the size of its hash region.
// clev[c] becomes the cloud's node count per level (0 below its lmin).
__global__ void k_cloud_levels(int nc, int32_t *__restrict__ clev, GridParams *__restrict__ P, float budget)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    int32_t *cl = clev + (int64_t)c * kLevels;
    int32_t cnt[kLevels];
    int32_t run = 0;
    for (int l = kLevels - 1; l >= 0; l--) {
        run += cl[l];
        cnt[l] = run;           // points opening a cell at level >= l = cells at level l
    }
    int64_t n = P[c].n;
    int64_t cap = (int64_t)((double)budget * (double)n);
    if (cap < 1) cap = 1;
    int lmin = kLevels - 1;
    int64_t cum = 0;
    for (int l = kLevels - 1; l >= 0; l--) {
        cum += cnt[l];
        if (cum > cap) break;
        lmin = l;
    }
    int32_t nodes = 0;
    for (int l = 0; l < kLevels; l++) {
        cl[l] = (l >= lmin && n > 0) ? cnt[l] : 0;
        nodes += cl[l];
    }
    P[c].lmin = lmin;
    P[c].n_nodes = nodes;
    P[c].hash_cap = (uint32_t)(2 * nodes > 64 ? 2 * nodes : 64);
}

// Whole-grid layout: nodes per level summed over clouds, level offsets, and
// the hash regions of the clouds laid out one after another.
__global__ void __launch_bounds__(1024) k_layout(int nc, const int32_t *__restrict__ clev,
                                                 GridParams *__restrict__ P, GridLayout *__restrict__ L)
{
    __shared__ int32_t lsum[kLevels];
    __shared__ uint32_t wsum[16];
    __shared__ uint32_t carry;
    int t = threadIdx.x, w = t >> 6, lane = __lane_id();
    if (t < kLevels) lsum[t] = 0;
    if (t == 0) carry = 0;
    __syncthreads();
    for (int c0 = 0; c0 < nc; c0 += 1024) {
        int c = c0 + t;
        // level sums
        for (int l = 0; l < kLevels; l++) {
            int32_t v = c < nc ? clev[(int64_t)c * kLevels + l] : 0;
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
            if (lane == 0 && v) atomicAdd(&lsum[l], v);
        }
        // exclusive scan of hash region sizes
        uint32_t v = c < nc ? P[c].hash_cap : 0u, x = v;
        for (int o = 1; o < 64; o <<= 1) {
            uint32_t y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[w] = x;
        __syncthreads();
        uint32_t before = carry;
        for (int k = 0; k < w; k++) before += wsum[k];
        if (c < nc) P[c].hash_base = before + x - v;
        __syncthreads();
        if (t == 0) {
            uint32_t tot = 0;
            for (int k = 0; k < 16; k++) tot += wsum[k];
            carry += tot;
        }
        __syncthreads();
    }
    if (t == 0) {
        int32_t off = 0;
        for (int l = 0; l < kLevels; l++) {
            L->level_count[l] = lsum[l];
            L->level_off[l] = off;
            off += lsum[l];
        }
        L->n_nodes = off;
        L->hash_slots = carry;
    }
}

__device__ inline int point_lmin(const GridParams *__restrict__ P, const uint64_t *__restrict__ keys, int64_t i,
                                 int64_t n)
{
    return i < n ? P[key_cloud(keys[i])].lmin : kLevels;
}

// per tile of kLvlTile sorted points: number of cells each level opens
__global__ void __launch_bounds__(kLvlThreads) k_level_count(const uint32_t *__restrict__ slev,
                                                           const uint64_t *__restrict__ keys, int64_t n,
                                                           const GridParams *__restrict__ P,
                                                           int32_t *__restrict__ lb)
{
    __shared__ int32_t c[kLevels];
    int t = threadIdx.x;
    if (t < kLevels) c[t] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kLvlTile;
    for (int r = 0; r < kLvlItems; r++) {
        int64_t i = base + r * kLvlThreads + t;
        uint32_t s = (i < n) ? slev[i] : kNoStart;
        int lmin = (s != kNoStart) ? point_lmin(P, keys, i, n) : kLevels;
#pragma unroll
        for (int l = 0; l < kLevels; l++) {
            uint64_t b = __ballot(s != kNoStart && (int)s >= l && l >= lmin);
            if (__lane_id() == 0 && b) atomicAdd(&c[l], __popcll(b));
        }
    }
    __syncthreads();
    if (t < kLevels) lb[(int64_t)blockIdx.x * kLevels + t] = c[t];
}

// exclusive scan over tiles, one wave per level
__global__ void __launch_bounds__(1024) k_level_scan(int32_t *__restrict__ lb, int nblk)
{
    const int w = threadIdx.x >> 6;
    for (int l = w; l < kLevels; l += 16) wave_excl_scan(lb + l, kLevels, nblk);
}

// writes node starts, levels and first children
__global__ void __launch_bounds__(kLvlThreads) k_level_scatter(const uint32_t *__restrict__ slev,
                                                             const uint64_t *__restrict__ keys, int64_t n,
                                                             const GridParams *__restrict__ P,
                                                             const GridLayout *__restrict__ L,
                                                             const int32_t *__restrict__ lb,
                                                             Node *__restrict__ nodes)
{
    constexpr int W = kLvlThreads / 64;
    __shared__ int32_t running[kLevels];
    __shared__ int32_t wtot[kLevels][W];
    int t = threadIdx.x, w = t >> 6;
    if (t < kLevels) running[t] = lb[(int64_t)blockIdx.x * kLevels + t];
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kLvlTile;
    uint64_t lt = lanemask_lt();
    for (int r = 0; r < kLvlItems; r++) {
        int64_t i = base + r * kLvlThreads + t;
        uint32_t s = (i < n) ? slev[i] : kNoStart;
        int lmin = (s != kNoStart) ? point_lmin(P, keys, i, n) : kLevels;
        int32_t rank[kLevels];
#pragma unroll
        for (int l = 0; l < kLevels; l++) {
            bool f = s != kNoStart && (int)s >= l && l >= lmin;
            uint64_t b = __ballot(f);
            rank[l] = __popcll(b & lt);
            if (__lane_id() == 0) wtot[l][w] = __popcll(b);
        }
        __syncthreads();
        int32_t prev = -1;
#pragma unroll
        for (int l = 0; l < kLevels; l++) {
            bool f = s != kNoStart && (int)s >= l && l >= lmin;
            int32_t pos = running[l] + rank[l];
            for (int x = 0; x < w; x++) pos += wtot[l][x];
            int32_t node = L->level_off[l] + pos;
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
        if (t < kLevels) {
            int32_t s2 = 0;
            for (int x = 0; x < W; x++) s2 += wtot[t][x];
            running[t] += s2;
        }
        __syncthreads();
    }
}

__global__ void k_hash_clear(const GridLayout *__restrict__ L, HSlot *__restrict__ hs, int64_t cap_max)
{
    int64_t cap = L->hash_slots < cap_max ? L->hash_slots : cap_max;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cap; i += (int64_t)gridDim.x * blockDim.x)
        hs[i].key = kEmptyKey;
}

// node counts, child counts, hash insertion.  A node's run ends at the next
// node of its level or at the end of its cloud; its children are the nodes
// of the level below that start inside its run (at most 8, contiguous).
__global__ void k_nodes_finish(const GridParams *__restrict__ P, const GridLayout *__restrict__ L,
                               const uint64_t *__restrict__ keys, Node *__restrict__ nodes, HSlot *__restrict__ hs)
{
    int32_t total = L->n_nodes;
    for (int32_t m = blockIdx.x * blockDim.x + threadIdx.x; m < total; m += gridDim.x * blockDim.x) {
        // start, first_child and the level were written by the scatter pass
        // and are only read here; each thread writes its own node's counts
        uint32_t start = nodes[m].h.start;
        uint32_t meta = nodes[m].h.meta;
        int l = (int)(meta >> 8);
        int c = key_cloud(keys[start]);
        const GridParams &p = P[c];
        uint32_t cend = (uint32_t)(p.base + p.n);
        int32_t lend = L->level_off[l] + L->level_count[l];
        uint32_t next_start = (m + 1 < lend) ? nodes[m + 1].h.start : cend;
        uint32_t end = next_start < cend ? next_start : cend;
        nodes[m].h.count = end - start;
        if (l > p.lmin) {
            uint32_t fc = nodes[m].h.first_child;
            int32_t cend_lvl = L->level_off[l - 1] + L->level_count[l - 1];
            uint32_t nc = 1;
            while (nc < 8 && (int32_t)(fc + nc) < cend_lvl && nodes[fc + nc].h.start < end) nc++;
            nodes[m].h.meta = meta | nc;
        }
        uint64_t key = hash_key(l, (keys[start] & ((1ull << kCloudShift) - 1)) >> (3 * l));
        HSlot *region = hs + p.hash_base;
        uint32_t s = hash_slot(key, p.hash_cap);
        for (uint32_t it = 0; it < p.hash_cap; it++) {
            unsigned long long prev = atomicCAS((unsigned long long *)&region[s].key, (unsigned long long)kEmptyKey,
                                                (unsigned long long)key);
            if (prev == kEmptyKey) {
                region[s].val = (uint32_t)m;
                break;
            }
            s = next_slot(s, p.hash_cap);
        }
    }
}

// tight float32 boxes of the level-l nodes: from their points at their
// cloud's finest level, from their children's boxes above it
__global__ void k_node_boxes(const GridParams *__restrict__ P, const GridLayout *__restrict__ L, int l,
                             const uint64_t *__restrict__ keys, const float4 *__restrict__ pts, Node *__restrict__ nodes)
{
    int32_t off = L->level_off[l], end = off + L->level_count[l];
    for (int32_t m = off + blockIdx.x * blockDim.x + threadIdx.x; m < end; m += gridDim.x * blockDim.x) {
        NodeHdr h = nodes[m].h;
        float lx = INFINITY, ly = INFINITY, lz = INFINITY, hx = -INFINITY, hy = -INFINITY, hz = -INFINITY;
        if (l == P[key_cloud(keys[h.start])].lmin) {
            for (uint32_t j = h.start; j < h.start + h.count; j++) {
                float4 p = pts[j];
                lx = fminf(lx, p.x); ly = fminf(ly, p.y); lz = fminf(lz, p.z);
                hx = fmaxf(hx, p.x); hy = fmaxf(hy, p.y); hz = fmaxf(hz, p.z);
            }
        } else {
            uint32_t nc = node_nchild(h);
            for (uint32_t c = 0; c < nc; c++) {
                const Node &ch = nodes[h.first_child + c];
                lx = fminf(lx, ch.lo[0]); ly = fminf(ly, ch.lo[1]); lz = fminf(lz, ch.lo[2]);
                hx = fmaxf(hx, ch.hi[0]); hy = fmaxf(hy, ch.hi[1]); hz = fmaxf(hz, ch.hi[2]);
            }
        }
        Node &o = nodes[m];
        o.lo[0] = lx; o.lo[1] = ly; o.lo[2] = lz;
        o.hi[0] = hx; o.hi[1] = hy; o.hi[2] = hz;
        o.pad[0] = o.pad[1] = 0u;
    }
}

inline int blocks_for(int64_t n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

int64_t max_pyramid_nodes(int64_t n, int n_clouds)
{
    // each cloud keeps at most max(n_c, 1) nodes
    return n + n_clouds + 1;
}

void grid_carve(Carver &c, int64_t n, int n_clouds, GridStore &g)
{
    int64_t nn = n > 0 ? n : 1;
    int nc = n_clouds > 0 ? n_clouds : 1;
    g.n = n;
    g.n_clouds = nc;
    g.nblk_sort = (int)((nn + kSortTile - 1) / kSortTile);
    g.nblk_lvl = (int)((nn + kLvlTile - 1) / kLvlTile);
    g.max_nodes = max_pyramid_nodes(nn, nc);
    // a cloud's region holds max(64, 2 x its nodes) slots
    g.hash_slots_max = 2 * g.max_nodes + 64 * (int64_t)nc;
    g.node_budget = 1.0f;
    g.leaf = 16;
    g.params = c.take<GridParams>(nc);
    g.layout = c.take<GridLayout>(1);
    g.off = c.take<int64_t>(nc + 1);
    g.clev = c.take<int32_t>((size_t)nc * kLevels);
    g.bbox = c.take<uint32_t>((size_t)nc * 6);
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
    g.hash = c.take<HSlot>(g.hash_slots_max);
}

void grid_carve_sort(Carver &c, int64_t n, int n_clouds, GridStore &g)
{
    int64_t nn = n > 0 ? n : 1;
    int nc = n_clouds > 0 ? n_clouds : 1;
    g = GridStore{};
    g.n = n;
    g.n_clouds = nc;
    g.nblk_sort = (int)((nn + kSortTile - 1) / kSortTile);
    g.node_budget = 1.0f;
    g.leaf = 16;
    g.params = c.take<GridParams>(nc);
    g.off = c.take<int64_t>(nc + 1);
    g.clev = c.take<int32_t>((size_t)nc * kLevels);
    g.bbox = c.take<uint32_t>((size_t)nc * 6);
    g.keys = c.take<uint64_t>(nn);
    g.keys_alt = c.take<uint64_t>(nn);
    g.idx = c.take<uint32_t>(nn);
    g.idx_alt = c.take<uint32_t>(nn);
    g.pts = c.take<float4>(nn);
    g.radix_hist = c.take<uint32_t>((size_t)g.nblk_sort * kRadix);
    g.radix_tot = c.take<uint32_t>(kRadix);
}

size_t grid_bytes(int64_t n, int n_clouds)
{
    Carver c(nullptr, ~(size_t)0 >> 1);
    GridStore g;
    grid_carve(c, n, n_clouds, g);
    return c.used();
}

hipError_t grid_set_single_cloud(GridStore &g, hipStream_t s)
{
    k_single_cloud<<<1, 1, 0, s>>>(g.off, g.n);
    return hipGetLastError();
}

hipError_t grid_sort_points(GridStore &g, const float *xyz, hipStream_t s)
{
    const int64_t n = g.n;
    const int nc = g.n_clouds;
    const int T = 256;
    int ib = blocks_for((int64_t)nc * kLevels, T);
    k_cloud_init<<<ib < 1024 ? ib : 1024, T, 0, s>>>(nc, g.bbox, g.clev);
    int bb_blocks = blocks_for(n, kBoxTile);
    if (bb_blocks > 1024) bb_blocks = 1024;
    if (bb_blocks < 1) bb_blocks = 1;
    k_bbox<<<bb_blocks, T, 0, s>>>(xyz, g.off, nc, g.bbox);
    k_params<<<blocks_for(nc, T), T, 0, s>>>(g.bbox, g.off, nc, g.params);
    if (n > 0) {
        k_keys<<<blocks_for(n, T), T, 0, s>>>(xyz, g.off, nc, g.params, g.keys);
        // a single cloud needs the 48 Morton bits only; a batch also sorts by
        // the cloud index above them, one more pass per byte it needs
        int cloud_bits = 0;
        while (cloud_bits < 16 && (1 << cloud_bits) < nc) cloud_bits++;
        const int passes = (kCloudShift + cloud_bits + kRadixBits - 1) / kRadixBits;
        uint64_t *ka = g.keys, *kb = g.keys_alt;
        uint32_t *ia = nullptr, *ib2 = g.idx_alt;
        for (int p = 0; p < passes; p++) {
            int shift = p * kRadixBits;
            k_radix_hist<<<g.nblk_sort, kSortThreads, 0, s>>>(ka, n, shift, g.radix_hist);
            k_radix_colscan<<<kRadix / 4, 256, 0, s>>>(g.radix_hist, g.nblk_sort, g.radix_tot);
            k_radix_scatter<<<g.nblk_sort, kSortThreads, 0, s>>>(ka, ia, n, shift, g.radix_hist, g.radix_tot,
                                                                 kb, ib2);
            // ping-pong between the two buffers
            uint64_t *tk = ka; ka = kb; kb = tk;
            if (p == 0) { ia = g.idx_alt; ib2 = g.idx; }
            else { uint32_t *ti = ia; ia = ib2; ib2 = ti; }
        }
        // the sorted keys and indices are in (ka, ia): after an odd number of
        // passes that is the alternate pair, which then takes the primary
        // role (the alternates are used by the sort alone)
        g.keys = ka;
        g.keys_alt = kb;
        g.idx = ia;
        g.idx_alt = ib2;
        k_gather_pts<<<blocks_for(n, T), T, 0, s>>>(xyz, g.idx, n, g.pts);
    }
    return hipGetLastError();
}

namespace {

__global__ void k_pack_pts(const float *__restrict__ xyz, int64_t n, float4 *__restrict__ pts)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        pts[i] = make_float4(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], __uint_as_float((uint32_t)i));
}

}  // namespace

hipError_t grid_pack_points(GridStore &g, const float *xyz, hipStream_t s)
{
    if (g.n > 0) {
        int b = blocks_for(g.n, 256);
        k_pack_pts<<<b < 4096 ? b : 4096, 256, 0, s>>>(xyz, g.n, g.pts);
    }
    return hipGetLastError();
}

hipError_t grid_build(GridStore &g, const float *xyz, hipStream_t s)
{
    const int64_t n = g.n;
    const int nc = g.n_clouds;
    const int T = 256;
    hipError_t e = grid_sort_points(g, xyz, s);
    if (e != hipSuccess) return e;
    if (n > 0) k_slev<<<blocks_for(n, T), T, 0, s>>>(g.keys, n, g.slev, g.clev);
    float budget = g.node_budget > 0.f && g.node_budget <= 1.f ? g.node_budget : 1.f;
    k_cloud_levels<<<blocks_for(nc, T), T, 0, s>>>(nc, g.clev, g.params, budget);
    k_layout<<<1, 1024, 0, s>>>(nc, g.clev, g.params, g.layout);
    if (n > 0) {
        k_level_count<<<g.nblk_lvl, kLvlThreads, 0, s>>>(g.slev, g.keys, n, g.params, g.level_block);
        k_level_scan<<<1, 1024, 0, s>>>(g.level_block, g.nblk_lvl);
        k_level_scatter<<<g.nblk_lvl, kLvlThreads, 0, s>>>(g.slev, g.keys, n, g.params, g.layout, g.level_block,
                                                           g.node);
        int hb = blocks_for(g.hash_slots_max, T);
        if (hb > 4096) hb = 4096;
        k_hash_clear<<<hb, T, 0, s>>>(g.layout, g.hash, g.hash_slots_max);
        int nb = blocks_for(g.max_nodes, T);
        if (nb > 4096) nb = 4096;
        k_nodes_finish<<<nb, T, 0, s>>>(g.params, g.layout, g.keys, g.node, g.hash);
        int bxb = blocks_for(n, T);
        if (bxb > 2048) bxb = 2048;
        for (int l = 0; l < kLevels; l++)
            k_node_boxes<<<bxb, T, 0, s>>>(g.params, g.layout, l, g.keys, g.pts, g.node);
    }
    return hipGetLastError();
}

}  // namespace pcg
