// Host interface of the ICP kernels (icp.hip), used by the C-ABI layer.
#pragma once

#include "common.h"

namespace pcg {

struct IcpState;

// One ICP call over np pairs (np = 1 for icp_point_to_plane).  Source points
// of pair p are [soff[p], soff[p+1]) of the source array, target points are
// the grid's cloud p.  Every block of the accumulate kernel belongs to one
// pair: pair p owns blocks [boff[p], boff[p+1]) and reduction groups
// [goff[p], goff[p+1]).
struct IcpStore {
    GridStore grid;     // pyramid over the targets, one cloud per pair
    GridStore ssrc;     // the sources sorted by Morton key per pair (nearest association)
    float4 *nrm;        // target normals in sorted order; w: nearest-other-point gap (squared)
    int2 *prev;         // per source point: previous match (sorted position, node) or -1
    IcpState *st;       // per pair: pose and loop state
    int64_t *soff;      // source offsets (np + 1)
    int32_t *boff;      // block offsets (np + 1)
    int32_t *goff;      // reduction group offsets (np + 1)
    float *dmax;        // per pair: rejection distance
    int32_t *maxit;     // per pair: iteration limit
    float2 *part;       // per block: compensated partial sums
    uint32_t *pcnt;     // per block: inlier counts
    float2 *gpart;      // per group of blocks: merged partial sums
    uint32_t *gcnt;     // per group of blocks: inlier counts
    double *hist;       // per pair and iteration: increment, inliers, sum r^2
    int32_t *queue;     // persistent loop: tile counter per pass
    int hist_stride;    // doubles per pair in hist
    int np, nblk, ngrp, iters_max;
    int max_pair_groups;  // most reduction groups of any pair (small: the solve kernel merges them)
    int threads;        // accumulate block size (64, 128 or 256)
    int leaf;           // largest node scanned as a leaf by the search (8, 16 or 32)
    int metric;         // 0 point-to-plane, 1 point-to-point (closed form), 2 combined
    float w_point, w_plane;   // weights of the combined metric
    int assoc;          // kAssocNearest (grid search) or kAssocProjective (organized target)
    const float *ptgt, *pnrm;  // projective: organized target points and normals (height * width, 3)
    int width, height;
    float K[4];         // projective: fx, fy, cx, cy
    bool grid_built;    // the target pyramid is already built (by the caller, e.g. for its normals)
    bool nrm_ready;     // nrm already holds the sorted normals and gaps (written with the normals)
    bool sort_src;      // nearest association: visit the sources in Morton order (else input order)
    bool persistent;    // point-to-plane with nearest association: the whole loop in one cooperative launch
};

enum { kAssocNearest = 0, kAssocProjective = 1 };

// blocks of the accumulate kernel for ns source points with `threads` per
// block (icp_blocks_max: the smallest block size, which sizes the
// workspace); groups for nblk blocks
int64_t icp_blocks(int64_t ns, int threads);
int64_t icp_blocks_max(int64_t ns);
int64_t icp_groups(int64_t nblk);
void icp_carve(Carver &c, int np, int64_t ns, int64_t nt, int64_t nblk, int64_t ngrp, int iters_max,
               IcpStore &s);
// device-side layout of a single pair (offsets, blocks, groups, parameters)
hipError_t icp_layout_single(IcpStore &s, int64_t ns, int64_t nt, float dmax, int max_iters, hipStream_t st);
// Runs iters_max passes (pairs stop at their own limit) plus the final
// statistics pass.  The layout arrays must already be on the device.
hipError_t icp_run(IcpStore &s, const float *src, int64_t ns, const float *tgt, const float *tgt_n,
                   const double *init_T, double conv_tol, double *out_T, pc_icp_stats *out_stats, hipStream_t st);

void icp_set_timer(hipEvent_t *b, hipEvent_t *e, int cap);
int icp_timer_count();
// events around the search kernel of knn_run / normals_run (slot 0)
void timer_search_begin(hipStream_t st);
void timer_search_end(hipStream_t st);
// events of slot `slot` (ignored beyond the registered capacity)
void timer_slot_begin(int slot, hipStream_t st);
void timer_slot_end(int slot, hipStream_t st);

hipError_t knn_run(const GridStore &g, const float *qry, int64_t nq, int k, int32_t *oi, float *od, hipStream_t s);
// k_max: the largest k of any cloud; kc: per-cloud k (device), or null to
// use k_max for all; cap2: inclusive key limit of neighbours (hybrid), with
// fewer than min_pts neighbours giving normal 0
// srt (optional, plain k-NN only): the normals in sorted order with the
// nearest-other-point gap in w, as the ICP correspondence search reads them
hipError_t normals_run(const GridStore &g, const float *xyz, int k_max, const int32_t *kc, const float *vp,
                       float *on, float *oc, hipStream_t s, float cap2 = INFINITY, int min_pts = 0,
                       float4 *srt = nullptr);
// radius neighbourhoods: every point with key <= r2
hipError_t normals_radius_run(const GridStore &g, float r2, const float *vp, float *on, float *oc, hipStream_t s);

}  // namespace pcg
