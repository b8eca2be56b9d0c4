// Parameter layout and host interface of the learned pose initialiser and
// of the device side of multi-start ICP (pose_net.hip), used by the C-ABI
// layer.
#pragma once

#include "common.h"
#include "pcgpu.h"

namespace pcg {

constexpr int kC1 = 64, kC2 = 128, kC3 = 256, kH = 256;
constexpr int kStarts = 8;      // multi-start ICP: identity + 7 rotations
// flat float32 parameters, row-major matrices W[in][out]:
// W1 3x64, b1, W2 64x128, b2, W3 128x256, b3, W4 512x256, b4, W5 256x4, b5
// (each W followed by its b, so [W; b] is a row-major (in + 1) x out block)
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + 3 * kC1;
constexpr int kOffW2 = kOffB1 + kC1;
constexpr int kOffB2 = kOffW2 + kC1 * kC2;
constexpr int kOffW3 = kOffB2 + kC2;
constexpr int kOffB3 = kOffW3 + kC2 * kC3;
constexpr int kOffW4 = kOffB3 + kC3;
constexpr int kOffB4 = kOffW4 + 2 * kC3 * kH;
constexpr int kOffW5 = kOffB4 + kH;
constexpr int kOffB5 = kOffW5 + kH * 4;
constexpr int kParams = kOffB5 + 4;

struct PoseNetStore {
    int np, nc;                 // pairs and clouds (cloud 2p: source p, 2p + 1: target p)
    int ntile;                  // encoder tiles
    int nchunk;                 // outer-product chunks (training)
    int64_t *offs;              // the pairs' row offsets as uploaded: source (np + 1), then target (np + 1)
    int64_t *cr;                // per cloud: first and end row in its buffer (2 nc)
    int32_t *toff;              // tile offsets (nc + 1)
    double *cen;                // per cloud centroid
    float *scale;               // per cloud inverse RMS radius
    __bf16 *w3t;                // bfloat16 copy of W3, [n][k]
    __bf16 *w3p;                // W3 in the forward's K-slot order, [n][slot]
    __bf16 *w2p;                // W2 in the forward's K-slot order, [n][slot]
    __bf16 *w2q;                // W2 by rows, columns in that slot order, [j][slot]
    float *pmax;                // per tile x channel maxima
    int32_t *parg;              // ... and their point indices
    float *feat;                // per cloud features
    int32_t *arg;               // per cloud arg-max points
    float *z4, *q;              // per pair head pre-activations and quaternion
    double *T;                  // per pair predicted pose (when no output is given)
    // training only
    float *grad, *loss, *dq, *dz, *df;
    float *U1, *V1, *U2, *V2, *A2, *G3, *part;
};

int pose_net_tiles(int64_t n_cloud);
// carve for np pairs and ntile encoder tiles; train adds the backward buffers
void pose_net_carve(Carver &c, int np, int ntile, bool train, PoseNetStore &s);
// cr and toff from the offsets in s.offs (on the device)
hipError_t pose_net_layout(PoseNetStore &s, hipStream_t st);
// centroids and scales only (cr and toff must be on the device)
hipError_t pose_net_stats(PoseNetStore &s, const float *xs, const float *xt, hipStream_t st);
// forward: initial pose per pair into out_T (n_pairs x 16), or into s.T
// enc_slot >= 0: kernel timer slot recorded around the encoder kernel
hipError_t pose_net_forward(PoseNetStore &s, const float *params, const float *xs, const float *xt, double *out_T,
                            hipStream_t st, int enc_slot = -1);
// forward + weighted loss + backward (gradient into s.grad) + Adam step when lr > 0
hipError_t pose_net_train(PoseNetStore &s, float *params, float *adam_m, float *adam_v, int step, float lr,
                          const float *xs, const float *xt, const double *label_T, const float *pair_w,
                          float *out_loss, hipStream_t st);
// kStarts poses per listed pair, about the centroids in cen
hipError_t multi_start_poses(const double *cen, const int32_t *sel, int nsel, double *out_T, hipStream_t st);
// best start per listed pair into out_T / out_stats / out_start at the pair's index
hipError_t multi_start_select(const double *T_all, const pc_icp_stats *st_all, const int32_t *sel, int nsel,
                              double *out_T, pc_icp_stats *out_stats, int32_t *out_start, hipStream_t st);
hipError_t gather_rows3(const float *in, float *out, const int64_t *seg, int nseg, hipStream_t st);
hipError_t fill_i32(int32_t *p, int n, int32_t v, hipStream_t st);

}  // namespace pcg
