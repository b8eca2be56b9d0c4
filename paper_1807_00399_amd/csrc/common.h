// Internal definitions shared by the gfx950 kernels of the point-cloud
// library: the sparse voxel pyramid ("grid") layout, Morton keys, the cell
// hash and small device helpers.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pcgpu.h"

namespace pcg {

// ---------------------------------------------------------------------------
// Grid geometry.  The bounding cube of a cloud is split into 2^16 cells per
// axis (level 0).  A level-L cell groups 2^L x 2^L x 2^L level-0 cells, so
// its key is the level-0 Morton key shifted right by 3L, and level 16 is the
// whole cube.  Points are stored sorted by level-0 Morton key, which makes
// every cell at every level a contiguous run of the sorted array.
//
// One grid can hold a batch of clouds: the sort key is (cloud << 48 | Morton
// key), so each cloud is a contiguous run of the sorted array with its own
// cube, its own finest level and its own region of the cell hash.
// ---------------------------------------------------------------------------
constexpr int kBits = 16;                 // bits per axis at level 0
constexpr int kLevels = kBits + 1;        // levels 0..16
constexpr uint32_t kMaxCoord = (1u << kBits) - 1u;
constexpr uint64_t kEmptyKey = ~0ull;     // empty hash slot

constexpr int kCloudShift = 48;           // cloud index position in sort keys

struct GridParams {        // one per cloud, written on the device by the grid builder
    float ox, oy, oz;      // origin (cube corner)
    float inv_h0;          // 1 / level-0 cell width
    float h0;              // level-0 cell width
    float margin;          // absolute slack for cell-range tests (a few ulps of the extent)
    int32_t n;             // points of this cloud
    int32_t base;          // its first position in the sorted arrays
    int32_t lmin;          // finest level kept for this cloud
    int32_t n_nodes;       // nodes of this cloud
    uint32_t hash_base;    // first slot of its hash region
    uint32_t hash_cap;     // slots of its hash region (at least twice its nodes)
};

struct GridLayout {        // whole grid, written on the device by the grid builder
    int32_t level_count[kLevels];   // nodes per level, all clouds
    int32_t level_off[kLevels];     // first node of each level in the node array
    int32_t n_nodes;       // total nodes
    uint32_t hash_slots;   // total hash slots in use
};

// Node header: start/count of its run in the sorted arrays, first child
// (global node index, level L-1) and meta = number of children | level << 8.
struct NodeHdr {
    uint32_t start, count, first_child, meta;
};
__host__ __device__ inline uint32_t node_nchild(const NodeHdr &h) { return h.meta & 0xffu; }
__host__ __device__ inline int node_level(const NodeHdr &h) { return (int)(h.meta >> 8); }

// One 48-byte node record: header plus the tight float32 box of the node's
// points (the minimum and maximum of their coordinates).  One load brings
// everything a traversal step needs.
struct Node {
    NodeHdr h;
    float lo[3], hi[3];
    uint32_t pad[2];
};

// Hash slot: (level << 48 | cell key) and node index in one 16-byte load.
struct HSlot {
    uint64_t key;
    uint32_t val, pad;
};

// Views of the workspace the grid lives in.
struct GridView {
    const GridParams *params;  // per cloud
    const float4 *pts;         // sorted points; .w = original index (bit pattern)
    const uint64_t *keys;      // sorted (cloud << 48 | level-0 Morton key)
    const Node *node;
    const HSlot *hash;
};

// ---------------------------------------------------------------------------
// Morton keys
// ---------------------------------------------------------------------------
__host__ __device__ inline uint64_t spread3(uint32_t v)
{
    uint64_t x = v & 0xffffu;
    x = (x | (x << 16)) & 0x0000ff0000ffull;
    x = (x | (x << 8)) & 0x00f00f00f00full;
    x = (x | (x << 4)) & 0x0c30c30c30c3ull;
    x = (x | (x << 2)) & 0x249249249249ull;
    return x;
}

__host__ __device__ inline uint32_t compact3(uint64_t x)
{
    x &= 0x249249249249ull;
    x = (x | (x >> 2)) & 0x0c30c30c30c3ull;
    x = (x | (x >> 4)) & 0x00f00f00f00full;
    x = (x | (x >> 8)) & 0x0000ff0000ffull;
    x = (x | (x >> 16)) & 0xffffull;
    return (uint32_t)x;
}

__host__ __device__ inline uint64_t morton3(uint32_t x, uint32_t y, uint32_t z)
{
    return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

__device__ inline uint64_t hash_key(int level, uint64_t cellkey)
{
    return ((uint64_t)level << 48) | cellkey;
}

// home slot of a key in a region of `cap` slots: the two 32-bit halves
// mixed by multiplications and xor-shifts (32-bit arithmetic only), then
// scaled to [0, cap) (no power-of-two size)
__device__ inline uint32_t hash_slot(uint64_t k, uint32_t cap)
{
    uint32_t h = (uint32_t)k * 0x9e3779b1u ^ ((uint32_t)(k >> 32) + 0x7f4a7c15u) * 0x85ebca77u;
    h ^= h >> 15;
    h *= 0x2c1b3c6du;
    h ^= h >> 12;
    h *= 0x297a2d39u;
    h ^= h >> 15;
    return (uint32_t)(((uint64_t)h * cap) >> 32);
}

// Morton key of the cell one step up along x (axis 0), y (1) or z (2):
// the axis bits are incremented in place (dilated-integer addition)
template <int AXIS>
__device__ inline uint64_t morton_inc(uint64_t m)
{
    constexpr uint64_t mask = 0x249249249249ull << AXIS;
    return (m & ~mask) | (((m | ~mask) + (1ull << AXIS)) & mask);
}

__device__ inline uint32_t next_slot(uint32_t s, uint32_t cap) { return (s + 1 == cap) ? 0u : s + 1; }

// Node index of cell (level, cx, cy, cz) of cloud P, or -1 when the cell is empty.
__device__ inline int32_t find_cell(const GridView &g, const GridParams &P, int level,
                                    uint32_t cx, uint32_t cy, uint32_t cz)
{
    uint64_t key = hash_key(level, morton3(cx, cy, cz));
    const HSlot *hs = g.hash + P.hash_base;
    uint32_t s = hash_slot(key, P.hash_cap);
    // the region is at most half full, so an empty slot ends every probe;
    // the bound only guards against a corrupted table
    for (uint32_t it = 0; it < P.hash_cap; it++) {
        HSlot e = hs[s];
        if (e.key == key) return (int32_t)e.val;
        if (e.key == kEmptyKey) return -1;
        s = next_slot(s, P.hash_cap);
    }
    return -1;
}

__host__ __device__ inline int key_cloud(uint64_t key) { return (int)(key >> kCloudShift); }

// cloud holding sorted position (or input index) i, for offsets off[0..nc]
__device__ inline int cloud_of(const int64_t *off, int nc, int64_t i)
{
    int lo = 0, hi = nc - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// float32 squared distance, the ranking key of the k-NN definition
__device__ inline float knn_key(float rx, float ry, float rz, float qx, float qy, float qz)
{
    float dx = rx - qx, dy = ry - qy, dz = rz - qz;
    return __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, __fmul_rn(dx, dx)));
}

// order-preserving float <-> uint mapping for atomic min/max
__device__ inline uint32_t f2ord(float f)
{
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float ord2f(uint32_t u)
{
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__device__ inline uint32_t lane_id() { return __lane_id(); }

// Squared distance from q to a box, evaluated like knn_key (per-axis
// differences, then fma in z, y, x order).  Rounding to nearest is monotone,
// so for every point p inside the box each rounded per-axis difference is at
// least the box's in magnitude and the result never exceeds knn_key(p, q):
// a box is skipped (distance > bound) only when every point in it is.
__device__ inline float box_key(float lx, float ly, float lz, float hx, float hy, float hz, float qx, float qy,
                                float qz)
{
    float dx = fmaxf(fmaxf(lx - qx, qx - hx), 0.f);
    float dy = fmaxf(fmaxf(ly - qy, qy - hy), 0.f);
    float dz = fmaxf(fmaxf(lz - qz, qz - hz), 0.f);
    return __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, __fmul_rn(dx, dx)));
}

__device__ inline float node_mindist2(const Node &nd, float qx, float qy, float qz)
{
    return box_key(nd.lo[0], nd.lo[1], nd.lo[2], nd.hi[0], nd.hi[1], nd.hi[2], qx, qy, qz);
}

// distance of node m from its box alone (24 of its 48 bytes)
__device__ inline float node_box_mindist2(const Node *node, uint32_t m, float qx, float qy, float qz)
{
    const char *r = reinterpret_cast<const char *>(node + m);
    const float4 a = *reinterpret_cast<const float4 *>(r + 16);   // lo x, y, z, hi x
    const float2 b = *reinterpret_cast<const float2 *>(r + 32);   // hi y, z
    return box_key(a.x, a.y, a.z, a.w, b.x, b.y, qx, qy, qz);
}

// Blocks are dispatched round-robin over the 8 XCDs, each with its own L2:
// map dispatch order so every XCD works on a contiguous range of queries,
// whose neighbourhoods overlap in its cache.  A bijection on [0, nblk).
__device__ inline int xcd_block(int b, int nblk)
{
    int full = (nblk / 8) * 8;
    return b < full ? (b % 8) * (nblk / 8) + b / 8 : b;
}

// Squared distance from q to the closed box of a grid cell, computed in
// float32 and shrunk so that it never exceeds the true distance of any point
// the cell holds (points are binned with the same rounding, see cell0).
__device__ inline float cell_mindist2(const GridParams &P, float qx, float qy, float qz,
                                      uint32_t cx, uint32_t cy, uint32_t cz, int level)
{
    float w = P.h0 * (float)(1u << level);
    float lx = P.ox + (float)cx * w, ly = P.oy + (float)cy * w, lz = P.oz + (float)cz * w;
    float dx = fmaxf(fmaxf(lx - qx, qx - (lx + w)), 0.f);
    float dy = fmaxf(fmaxf(ly - qy, qy - (ly + w)), 0.f);
    float dz = fmaxf(fmaxf(lz - qz, qz - (lz + w)), 0.f);
    dx = fmaxf(dx - P.margin, 0.f);
    dy = fmaxf(dy - P.margin, 0.f);
    dz = fmaxf(dz - P.margin, 0.f);
    return (dx * dx + dy * dy + dz * dz) * (1.0f - 1e-5f);
}

// level-0 cell coordinate of a coordinate value (clamped to the grid)
__device__ inline uint32_t cell0(float v, float o, float inv_h0)
{
    float c = floorf((v - o) * inv_h0);
    c = fminf(fmaxf(c, 0.f), (float)kMaxCoord);
    return (uint32_t)c;
}

// ---------------------------------------------------------------------------
// workspace carving
// ---------------------------------------------------------------------------
struct Carver {
    uintptr_t base, cur, end;
    bool ok;
    Carver(void *p, size_t bytes)
        : base((uintptr_t)p), cur((uintptr_t)p), end((uintptr_t)p + bytes), ok(true) {}
    template <class T>
    T *take(size_t count)
    {
        uintptr_t a = (cur + 255) & ~(uintptr_t)255;
        uintptr_t e = a + count * sizeof(T);
        if (e > end) ok = false;
        cur = e;
        return reinterpret_cast<T *>(a);
    }
    size_t used() const { return (size_t)(cur - base) + 256; }
};

// ---------------------------------------------------------------------------
// Grid storage inside a caller workspace and its builder (grid.hip)
// ---------------------------------------------------------------------------
struct GridStore {
    GridParams *params;       // per cloud
    GridLayout *layout;
    int64_t *off;             // cloud offsets into the input (n_clouds + 1)
    int32_t *clev;            // per cloud and level: slev histogram, then node counts
    uint64_t *keys, *keys_alt;
    uint32_t *idx, *idx_alt;
    float4 *pts;
    Node *node;
    HSlot *hash;
    uint32_t *slev;           // per sorted point: top level at which it starts a cell (or 0xff)
    uint32_t *radix_hist;     // radix histograms / scan space
    uint32_t *radix_tot;      // per-digit totals of a pass
    int32_t *level_block;     // per block, per level: counts then offsets
    uint32_t *bbox;           // per cloud: 6 ordered-uint min/max
    int64_t n;                // points of all clouds
    int n_clouds;
    int64_t max_nodes;
    int64_t hash_slots_max;
    float node_budget;        // nodes allowed per point when picking a cloud's finest level (<= 1)
    int leaf;                 // k-NN / normals searches scan nodes of at most this many points whole (8, 16, 32)
    int nblk_sort, nblk_lvl;
    GridView view() const
    {
        return GridView{params, pts, keys, node, hash};
    }
};

size_t grid_bytes(int64_t n, int n_clouds);
void grid_carve(Carver &c, int64_t n, int n_clouds, GridStore &g);
// the part of a grid store that sorting needs (grid_sort_points)
void grid_carve_sort(Carver &c, int64_t n, int n_clouds, GridStore &g);
// Sorts the points of every cloud by (cloud, Morton key of the cloud's
// cube) into g.pts (float4, .w = original index); g.off as for grid_build.
hipError_t grid_sort_points(GridStore &g, const float *xyz, hipStream_t s);
// The same points in input order into g.pts (.w = index).
hipError_t grid_pack_points(GridStore &g, const float *xyz, hipStream_t s);
// Builds the pyramid over xyz (n x 3 float32, device), clouds split by
// g.off (device, n_clouds + 1 entries, written by the caller beforehand or
// by grid_set_single_cloud).  Asynchronous.
hipError_t grid_build(GridStore &g, const float *xyz, hipStream_t s);
// Writes the offsets of a grid holding one cloud of g.n points.
hipError_t grid_set_single_cloud(GridStore &g, hipStream_t s);

int64_t max_pyramid_nodes(int64_t n, int n_clouds);

}  // namespace pcg
