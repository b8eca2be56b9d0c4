// Host interface of the ICP kernels (icp.hip), used by the C-ABI layer.
#pragma once

#include "common.h"

namespace pcg {

struct IcpState;

struct IcpStore {
    GridStore grid;     // pyramid over the target
    float4 *nrm;        // target normals in sorted order
    int2 *prev;         // per source point: previous match (sorted position, node) or -1
    IcpState *st;       // pose and loop state
    float2 *part;       // per block: compensated partial sums
    uint32_t *pcnt;     // per block: inlier counts
    float2 *gpart;      // per group of blocks: merged partial sums
    uint32_t *gcnt;     // per group of blocks: inlier counts
    int ngrp;
    double *hist;       // per iteration: increment, inliers, sum r^2
    int nblk, ppt;
};

void icp_carve(Carver &c, int64_t ns, int64_t nt, int max_iters, IcpStore &s);
hipError_t icp_run(IcpStore &s, const float *src, int64_t ns, const float *tgt, const float *tgt_n, int64_t nt,
                   const double *init_T, float dmax, int max_iters, double conv_tol, double *out_T,
                   pc_icp_stats *out_stats, hipStream_t st);

void icp_set_timer(hipEvent_t *b, hipEvent_t *e, int cap);
int icp_timer_count();

hipError_t knn_run(const GridStore &g, const float *qry, int64_t nq, int k, int32_t *oi, float *od, hipStream_t s);
hipError_t normals_run(const GridStore &g, const float *xyz, int k, const float *vp, float *on, float *oc,
                       hipStream_t s);

}  // namespace pcg
