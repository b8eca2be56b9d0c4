// Learned pose initialiser in front of ICP: a point-wise MLP encoder with a
// max-pool (per cloud) and a small head (per pair) that predicts the
// rotation; the translation aligns the centroids.  Also the pieces of
// multi-start ICP that run on the device: start poses, replication of the
// pairs that need them, and selection of the best start.
//
// Not part of the paper's method: its ICP starts from a given pose
// (Section 3, "Iterative geometric registration").  This network proposes
// that pose, batched ICP refines it, and pairs whose refinement does not
// reach a small residual fall back to multi-start ICP.
//
// Encoder per point (centred on the cloud centroid, scaled by the inverse
// RMS radius): 3 -> 64 (ReLU) -> 128 (ReLU) -> 256 (ReLU), then the
// per-channel maximum over the cloud's points.  The 64 -> 128 and
// 128 -> 256 layers are dense contractions over every point and run on the
// bfloat16 matrix cores (v_mfma_f32_16x16x32_bf16, float32 accumulation),
// with their inputs rounded to bfloat16; the first layer (3 inputs and the
// bias) runs on the float32 matrix cores (v_mfma_f32_16x16x4_f32); the head
// is float32 vector code.
//
// Training: the loss of a pair is w_p |R(q) - R_label|_F^2.  The max-pool
// routes each channel's gradient to one point, so the encoder's backward
// recomputes one row per (cloud, channel) instead of keeping activations of
// every point; the bfloat16 roundings pass gradients unchanged.  Weight
// gradients are sums over those rows (or over pairs) formed in a fixed order
// by chunked outer-product kernels (layer 2 on the bfloat16 matrix cores)
// and a second pass over the chunks: no atomics, so a step is deterministic.  Adam updates the float32 master
// parameters.

#include <math.h>

#include "common.h"
#include "icp.h"
#include "pose_net.h"

namespace pcg {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kT = 512;          // points per encoder tile
constexpr int kEncWaves = 8;     // waves per encoder workgroup; wave w owns rows 64w .. 64w + 63
constexpr int kEncThreads = 64 * kEncWaves;
constexpr int kP1 = kC1 + 8;     // padded LDS row lengths (bank spread)
constexpr int kP2 = kC2 + 8;
constexpr int kChunk = 128;      // rows per outer-product chunk

__device__ inline __bf16 to_bf16(float x) { return (__bf16)x; }

// ReLU of two float32 values rounded to bfloat16 and packed in one word (a
// packed conversion, then a packed signed 16-bit maximum with zero: a
// negative value, sign bit set, -0 included, becomes +0).  Rounding to
// nearest keeps the sign, so rounding first and clamping afterwards gives
// what clamping first would, at one instruction per two values for the
// clamp, where a float maximum in IEEE mode takes two per value (one quiets
// the operand).
__device__ inline uint32_t relu_pk_bf16(float a, float b)
{
    const bf16x2 h = __builtin_convertvector((f32x2){a, b}, bf16x2);
    const s16x2 r = __builtin_elementwise_max(__builtin_bit_cast(s16x2, h), (s16x2){0, 0});
    return __builtin_bit_cast(uint32_t, r);
}

// the four words of one accumulator tile's ReLU'd bfloat16 values
__device__ inline u32x2 relu_tile(f32x4 a) { return u32x2{relu_pk_bf16(a[0], a[1]), relu_pk_bf16(a[2], a[3])}; }

// two tiles' halves into one eight-value operand (lo in slots 0-3)
__device__ inline bf16x8 join_bf16x8(u32x2 lo, u32x2 hi)
{
    return __builtin_bit_cast(bf16x8, u32x4{lo[0], lo[1], hi[0], hi[1]});
}

// rows of cloud c: [cr[2c], cr[2c + 1]) of the source buffer (even c) or
// the target buffer (odd c)
__device__ inline const float *cloud_xyz(const float *xs, const float *xt, int c) { return (c & 1) ? xt : xs; }

// per cloud: centroid (float64) and inverse RMS radius
__global__ void k_norm_stats(const float *__restrict__ xs, const float *__restrict__ xt,
                             const int64_t *__restrict__ cr, int nc, double *__restrict__ cen,
                             float *__restrict__ scale)
{
    __shared__ double red[4][4];
    const int c = blockIdx.x;
    if (c >= nc) return;
    const float *X = cloud_xyz(xs, xt, c);
    const int64_t a = cr[2 * c], b = cr[2 * c + 1];
    double s[3] = {0.0, 0.0, 0.0};
    // unrolled so that several points' loads are in flight; each thread's
    // sums still take its points in ascending order
#pragma unroll 8
    for (int64_t i = a + threadIdx.x; i < b; i += blockDim.x)
        for (int k = 0; k < 3; k++) s[k] += X[3 * i + k];
    for (int o = 32; o > 0; o >>= 1)
        for (int k = 0; k < 3; k++) s[k] += __shfl_xor(s[k], o);
    const int w = threadIdx.x >> 6;
    if (__lane_id() == 0)
        for (int k = 0; k < 3; k++) red[w][k] = s[k];
    __syncthreads();
    const double n = (double)(b - a);
    double m[3];
    for (int k = 0; k < 3; k++) m[k] = n > 0 ? (red[0][k] + red[1][k] + red[2][k] + red[3][k]) / n : 0.0;
    double r2 = 0.0;
#pragma unroll 8
    for (int64_t i = a + threadIdx.x; i < b; i += blockDim.x)
        for (int k = 0; k < 3; k++) {
            double d = X[3 * i + k] - m[k];
            r2 += d * d;
        }
    for (int o = 32; o > 0; o >>= 1) r2 += __shfl_xor(r2, o);
    if (__lane_id() == 0) red[w][3] = r2;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < 3; k++) cen[3 * c + k] = m[k];
        double rms = n > 0 ? sqrt((red[0][3] + red[1][3] + red[2][3] + red[3][3]) / n) : 0.0;
        scale[c] = rms > 0.0 ? (float)(1.0 / rms) : 1.0f;
    }
}

// Layer 3 takes its K operand straight from layer 2's output registers,
// whose channel order per lane differs from the natural one: slot s of
// 32-wide k-block kb carries channel w3_slot_channel(kb, s).
__device__ inline int w3_slot_channel(int kb, int s)
{
    const int g = s >> 3, j = s & 7;
    return 32 * kb + (j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4));
}

// bfloat16 copies of the weights the matrix cores read: W3 with k
// contiguous per output column (w3t: [n][k]); W2 and W3 in the slot order of
// the forward (w2p: [n][slot], slot < 64; w3p: [n][slot], slot < 128); W2 by
// rows with its columns in that slot order (w2q: [j][slot], slot < 128)
__global__ void k_weights_bf16(const float *__restrict__ params, __bf16 *__restrict__ w3t, __bf16 *__restrict__ w3p,
                               __bf16 *__restrict__ w2p, __bf16 *__restrict__ w2q)
{
    const float *W2 = params + kOffW2, *W3 = params + kOffW3;
    constexpr int n3 = kC2 * kC3, n2 = kC1 * kC2;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 2 * n3 + 2 * n2; i += gridDim.x * blockDim.x) {
        if (i < n3) {
            const int n = i / kC2, k = i % kC2;
            w3t[i] = to_bf16(W3[k * kC3 + n]);
        } else if (i < 2 * n3) {
            const int q = i - n3, n = q / kC2, sl = q % kC2;
            w3p[q] = to_bf16(W3[w3_slot_channel(sl / 32, sl % 32) * kC3 + n]);
        } else if (i < 2 * n3 + n2) {
            const int q = i - 2 * n3, n = q / kC1, sl = q % kC1;
            w2p[q] = to_bf16(W2[w3_slot_channel(sl / 32, sl % 32) * kC2 + n]);
        } else {
            const int q = i - 2 * n3 - n2, jr = q / kC2, sl = q % kC2;
            w2q[q] = to_bf16(W2[jr * kC2 + w3_slot_channel(sl / 32, sl % 32)]);
        }
    }
}

// normalised coordinates of row i of cloud c
__device__ inline void norm_point(const float *X, int64_t i, const double *cen, float s, int c, float &x, float &y,
                                  float &z)
{
    x = (float)(X[3 * i] - cen[3 * c]) * s;
    y = (float)(X[3 * i + 1] - cen[3 * c + 1]) * s;
    z = (float)(X[3 * i + 2] - cen[3 * c + 2]) * s;
}

// Encoder forward.  Persistent workgroups (kEncWaves waves) load the
// bfloat16 weights into LDS once and then take a contiguous run of tiles of
// kT points (a tile holds points of one cloud).  Each lane keeps its
// running per-channel maximum over the tiles of one cloud in its own LDS
// slot, so tiles need no barrier; at a cloud's last tile in the run the
// slots are combined and the maximum activation per channel is written,
// with ARG (training) the lowest point index reaching it (without it, a
// point of the cloud stands in); the run's other tiles of that cloud are
// marked empty for the pool.
//
// Matrix-core operands of v_mfma_f32_16x16x32_bf16 (wave of 64 lanes, g =
// l / 16): lane l supplies A[l % 16][8 g + j] and B[8 g + j][l % 16] for
// j < 8 and receives C[4 g + i][l % 16] for i < 4.  Each wave owns 64 rows
// as four 16-row tiles m, and every weight fragment read from LDS feeds the
// four of them.
//   layer 2, transposed: C2^T[ch][row] = sum_k W2^T[ch][k] a1^T[k][row]; the
//     B operand (a1 of row l % 16, channels 32 kb + 8 g + j) is computed by
//     the lane itself from the point, so layer 1 never leaves registers;
//   the lane then holds channels 16 t + 4 g + i of row l % 16 (tiles t < 8),
//     which, paired as tiles (2 kb, 2 kb + 1), are the A operand of layer 3
//     in slot order (w3_slot_channel); W3 is stored in that order;
//   layer 3: C3[row][ch] = sum_k a2[row][k] W3[k][ch], 16 column tiles.
template <bool ARG>
__global__ void __launch_bounds__(kEncThreads) k_enc_forward(const float *__restrict__ xs, const float *__restrict__ xt,
                                                           const int64_t *__restrict__ cr,
                                                           const int32_t *__restrict__ toff, int nc, int ntile,
                                                           const double *__restrict__ cen,
                                                           const float *__restrict__ scale,
                                                           const float *__restrict__ params,
                                                           const __bf16 *__restrict__ w2p,
                                                           const __bf16 *__restrict__ w3p,
                                                           float *__restrict__ pmax, int32_t *__restrict__ parg)
{
    __shared__ __attribute__((aligned(16))) __bf16 sW2[kC2 * kP1];   // W2^T: [ch][slot], slot < 64
    __shared__ __attribute__((aligned(16))) __bf16 sW3[kC3 * kP2];   // W3: [n][slot], slot < 128
    __shared__ __attribute__((aligned(16))) float4 sW1[kC1];         // (w1x, w1y, w1z, b1) per channel
    __shared__ float sB2[kC2], sB3[kC3];
    // running maxima per wave and lane group g; rows kC3 + 16 apart, so
    // the four groups of a wave (16 consecutive columns each) fall on
    // disjoint halves of the 32 banks, two groups per half
    constexpr int kRow = kC3 + 16;
    __shared__ float sMax[4 * kEncWaves][kRow];
    __shared__ int32_t sArg[ARG ? 4 * kEncWaves : 1][kRow];    // arg-max rows only for training
    __shared__ float sFinMax[kC3];                   // upper half of the combine
    __shared__ int32_t sFinArg[ARG ? kC3 : 1];
    const int t = threadIdx.x, w = t >> 6, l = __lane_id();
    const int lr = l & 15, g = l >> 4;
    for (int i = t; i < kC2 * (kC1 / 8); i += kEncThreads) {
        int n = i / (kC1 / 8), k8 = i % (kC1 / 8);
        *reinterpret_cast<bf16x8 *>(&sW2[n * kP1 + 8 * k8]) = *reinterpret_cast<const bf16x8 *>(&w2p[n * kC1 + 8 * k8]);
    }
    for (int i = t; i < kC3 * (kC2 / 8); i += kEncThreads) {
        int n = i / (kC2 / 8), k8 = i % (kC2 / 8);
        *reinterpret_cast<bf16x8 *>(&sW3[n * kP2 + 8 * k8]) = *reinterpret_cast<const bf16x8 *>(&w3p[n * kC2 + 8 * k8]);
    }
    {
        const float *W1 = params + kOffW1, *b1 = params + kOffB1, *b2 = params + kOffB2, *b3 = params + kOffB3;
        for (int c = t; c < kC1; c += kEncThreads) sW1[c] = make_float4(W1[c], W1[kC1 + c], W1[2 * kC1 + c], b1[c]);
        for (int c = t; c < kC2; c += kEncThreads) sB2[c] = b2[c];
        for (int c = t; c < kC3; c += kEncThreads) sB3[c] = b3[c];
    }
    __syncthreads();
    const int r0 = 64 * w;
    // the tile's cloud and the raw coordinates of this lane's four rows;
    // the next tile's are loaded while the current one is computed
    auto cloud_of = [&](int tl) {
        int lo = 0, hi = nc - 1;      // the last cloud c with toff[c] <= tl
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (toff[mid] <= tl) lo = mid;
            else hi = mid - 1;
        }
        return lo;
    };
    auto load_rows = [&](int tl, int cl, float *px, float *py, float *pz) {
        const float *X = cloud_xyz(xs, xt, cl);
        const int64_t q0 = cr[2 * cl] + (int64_t)(tl - toff[cl]) * kT, qe = cr[2 * cl + 1];
#pragma unroll
        for (int m = 0; m < 4; m++) {
            const int64_t i = q0 + r0 + 16 * m + lr;
            const bool ok = i < qe;
            px[m] = ok ? X[3 * i] : 0.f;
            py[m] = ok ? X[3 * i + 1] : 0.f;
            pz[m] = ok ? X[3 * i + 2] : 0.f;
        }
    };
    // a contiguous run of tiles per workgroup; the tiles of one cloud within
    // it form a segment, whose maxima are combined once, at its last tile
    const int per = (ntile + (int)gridDim.x - 1) / (int)gridDim.x;
    const int t0 = blockIdx.x * per, t1 = min(ntile, t0 + per);
    int tile = t0;
    int c = tile < t1 ? cloud_of(tile) : 0;
    float px[4], py[4], pz[4];
    if (tile < t1) load_rows(tile, c, px, py, pz);
    for (; tile < t1; tile++) {
        const int tn = tile + 1;
        int cn = c;
        float nx[4], ny[4], nz[4];
        if (tn < t1) {
            while (cn + 1 < nc && toff[cn + 1] <= tn) cn++;
            load_rows(tn, cn, nx, ny, nz);
        }
        const bool fresh = tile == t0 || toff[c] == tile;     // first tile of the segment
        const bool flush = tn == t1 || cn != c;               // last tile of the segment
        const int64_t p0 = cr[2 * c] + (int64_t)(tile - toff[c]) * kT;
        const int64_t pend = cr[2 * c + 1];
        const int32_t pc0 = (int32_t)(p0 - cr[2 * c]);       // the tile's first point within its cloud
        // layer 1 on the float32 matrix cores (v_mfma_f32_16x16x4_f32: lane l
        // supplies A[l % 16][g] and B[g][l % 16], receives C[4 g + i][l % 16]),
        // transposed: C1^T[ch][row] = sum_k [W1; b1]^T[ch][k] [x y z 1]^T[k][row]
        // per 16-channel tile tc1 and 16-row tile m.  The lane ends up with
        // channels 16 tc1 + 4 g + i of row r0 + 16 m + lr; tiles (2 kb,
        // 2 kb + 1) are then the B operand of layer 2 in slot order
        // (w3_slot_channel), W2 being stored in that order.
        bf16x8 x1[4][2];
        {
            const float s = scale[c];
            const double cx = cen[3 * c], cy = cen[3 * c + 1], cz = cen[3 * c + 2];
            float bop[4];
#pragma unroll
            for (int m = 0; m < 4; m++) {
                const bool ok = p0 + r0 + 16 * m + lr < pend;
                const float x = ok ? (float)(px[m] - cx) * s : 0.f;
                const float y = ok ? (float)(py[m] - cy) * s : 0.f;
                const float z = ok ? (float)(pz[m] - cz) * s : 0.f;
                bop[m] = g == 0 ? x : (g == 1 ? y : (g == 2 ? z : 1.f));
            }
#pragma unroll
            for (int kb = 0; kb < kC1 / 32; kb++) {
                const float aop0 = reinterpret_cast<const float *>(sW1)[4 * (32 * kb + lr) + g];
                const float aop1 = reinterpret_cast<const float *>(sW1)[4 * (32 * kb + 16 + lr) + g];
#pragma unroll
                for (int m = 0; m < 4; m++) {
                    const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
                    const f32x4 a0 = __builtin_amdgcn_mfma_f32_16x16x4f32(aop0, bop[m], zero, 0, 0, 0);
                    const f32x4 a1 = __builtin_amdgcn_mfma_f32_16x16x4f32(aop1, bop[m], zero, 0, 0, 0);
                    x1[m][kb] = join_bf16x8(relu_tile(a0), relu_tile(a1));
                }
            }
        }
        // layer 2 (transposed): per 16-channel tile, bias, ReLU, bfloat16,
        // stored straight into the layer-3 A operands (tiles 2 kb, 2 kb + 1)
        bf16x8 x2[4][4];
        u32x2 half[4];     // the even tile's rounded outputs, until the odd one completes the operand
#pragma unroll
        for (int tc = 0; tc < kC2 / 16; tc++) {
            f32x4 acc[4];
            const f32x4 b2v = {sB2[16 * tc + 4 * g], sB2[16 * tc + 4 * g + 1], sB2[16 * tc + 4 * g + 2],
                               sB2[16 * tc + 4 * g + 3]};
#pragma unroll
            for (int m = 0; m < 4; m++) acc[m] = b2v;        // the bias starts the sum
#pragma unroll
            for (int kb = 0; kb < 2; kb++) {
                const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&sW2[(16 * tc + lr) * kP1 + 32 * kb + 8 * g]);
#pragma unroll
                for (int m = 0; m < 4; m++) acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, x1[m][kb], acc[m], 0, 0, 0);
            }
#pragma unroll
            for (int m = 0; m < 4; m++) {
                const u32x2 h = relu_tile(acc[m]);
                if (tc & 1) x2[m][tc >> 1] = join_bf16x8(half[m], h);
                else half[m] = h;
            }
        }
        // layer 3 and, per channel, the maximum over this lane's 16 rows
        // (ascending, first maximum kept; rows past the cloud's end, only in
        // a cloud's last tile, are excluded).  Bias and ReLU are monotone,
        // so both are applied after the maximum: the feature is unchanged,
        // and its arg-max matters only where it is positive, where it is the
        // arg-max of the pre-activation.
        const bool all_valid = p0 + r0 + 63 < pend;     // uniform over the wave
        // the next column tile's weight fragments are read from LDS while
        // the current one's products run
        bf16x8 bw[4];
#pragma unroll
        for (int kb = 0; kb < 4; kb++) bw[kb] = *reinterpret_cast<const bf16x8 *>(&sW3[lr * kP2 + 32 * kb + 8 * g]);
#pragma unroll 2
        for (int n3 = 0; n3 < kC3 / 16; n3++) {
            const int col = 16 * n3 + lr;
            // without training the slot holds the unbiased running maximum
            // (the bias is added at the combine: rounding is monotone, so
            // the maximum of the biased values is the biased maximum); it is
            // read here, ahead of the products, so the wait for it does not
            // also wait for the weight fragments read below
            const float old = ARG ? 0.f : sMax[4 * w + g][col];
            bf16x8 bn[4];
            const int n3n = n3 + 1 < kC3 / 16 ? n3 + 1 : n3;
#pragma unroll
            for (int kb = 0; kb < 4; kb++)
                bn[kb] = *reinterpret_cast<const bf16x8 *>(&sW3[(16 * n3n + lr) * kP2 + 32 * kb + 8 * g]);
            f32x4 acc[4];
#pragma unroll
            for (int m = 0; m < 4; m++) acc[m] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 4; kb++)
#pragma unroll
                for (int m = 0; m < 4; m++)
                    acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x2[m][kb], bw[kb], acc[m], 0, 0, 0);
#pragma unroll
            for (int kb = 0; kb < 4; kb++) bw[kb] = bn[kb];
            float best = -INFINITY;
            int32_t barg = 0x7fffffff;
            if (all_valid) {
                // NaN-propagating maximum: the matrix cores' finite outputs
                // need no quieting, and three operands go to one instruction
#pragma unroll
                for (int m = 0; m < 4; m++)
                    best = __builtin_elementwise_maximum(
                        __builtin_elementwise_maximum(best, __builtin_elementwise_maximum(acc[m][0], acc[m][1])),
                        __builtin_elementwise_maximum(acc[m][2], acc[m][3]));
                if (ARG) {
                    // the lowest of this lane's rows reaching it (rows in
                    // descending order, each equal one overwriting)
#pragma unroll
                    for (int m = 3; m >= 0; m--)
#pragma unroll
                        for (int i = 3; i >= 0; i--)
                            barg = acc[m][i] == best ? r0 + 16 * m + 4 * g + i : barg;
                } else {
                    barg = r0 + 4 * g;
                }
            } else {
#pragma unroll
                for (int m = 0; m < 4; m++)
#pragma unroll
                    for (int i = 0; i < 4; i++) {
                        const int row = r0 + 16 * m + 4 * g + i;
                        if (p0 + row < pend && acc[m][i] > best) { best = acc[m][i]; barg = row; }
                    }
            }
            // this lane's running maximum over the segment's tiles, in its
            // own LDS slot (no other lane touches it until the combine);
            // ties keep the earlier tile, whose rows are lower
            if (ARG) {
                const float v = best + sB3[col];
                const int32_t a = barg == 0x7fffffff ? barg : pc0 + barg;
                if (fresh || v > sMax[4 * w + g][col]) {
                    sMax[4 * w + g][col] = v;
                    sArg[4 * w + g][col] = a;
                }
            } else {
                sMax[4 * w + g][col] = fresh ? best : __builtin_elementwise_maximum(old, best);
            }
        }
        if (!flush) {
            // the segment's result goes to its last tile; the pool skips
            // the others
            if (t < kC3) parg[(int64_t)tile * kC3 + t] = -1;
        } else {
        __syncthreads();
        // across lanes and waves, ties to the lower row: each column's 32
        // partials in two halves of 16, one per thread
        static_assert(kEncThreads == 2 * kC3, "two threads per column");
        {
            const int col = t & (kC3 - 1), h = t / kC3;
            float best = -INFINITY;
            int32_t barg = 0x7fffffff;
#pragma unroll
            for (int x = 0; x < 2 * kEncWaves; x++) {
                const float v = sMax[2 * kEncWaves * h + x][col];
                if (ARG) {
                    const int32_t a = sArg[2 * kEncWaves * h + x][col];
                    if (v > best || (v == best && a < barg)) { best = v; barg = a; }
                } else if (v > best) {
                    best = v;
                }
            }
            if (h == 1) {
                sFinMax[col] = best;
                if (ARG) sFinArg[col] = barg;
            }
            __syncthreads();
            if (h == 0) {
                const float v = sFinMax[col];
                if (ARG) {
                    const int32_t a = sFinArg[col];
                    if (v > best || (v == best && a < barg)) { best = v; barg = a; }
                } else {
                    if (v > best) best = v;
                    // every tile has points, so every column a finite maximum;
                    // without training the index is not used, 0 marks it valid
                    barg = best == -INFINITY ? 0x7fffffff : 0;
                    best += sB3[col];
                }
                pmax[(int64_t)tile * kC3 + col] = fmaxf(best, 0.f);
                parg[(int64_t)tile * kC3 + col] = barg == 0x7fffffff ? -1 : barg;
            }
        }
        __syncthreads();
        }
#pragma unroll
        for (int m = 0; m < 4; m++) {
            px[m] = nx[m];
            py[m] = ny[m];
            pz[m] = nz[m];
        }
        c = cn;
    }
}

// The cloud layout from the pairs' row offsets (off: the source offsets
// 0..np, then the target offsets 0..np): rows [cr[2c], cr[2c + 1]) of cloud
// c (2p: source p, 2p + 1: target p), and toff, the exclusive prefix sum of
// the clouds' tile counts (toff[nc] = all tiles).  One workgroup, in chunks
// of 1024 clouds; integer sums, so the result is exact.
__global__ void __launch_bounds__(1024) k_pose_layout(const int64_t *__restrict__ off, int np,
                                                    int64_t *__restrict__ cr, int32_t *__restrict__ toff)
{
    __shared__ int32_t wsum[16];
    const int nc = 2 * np, t = threadIdx.x, w = t >> 6, l = __lane_id();
    int32_t carry = 0;     // tiles before this chunk (the same in every thread)
    for (int base = 0; base < nc; base += 1024) {
        const int c = base + t;
        int32_t v = 0;
        if (c < nc) {
            const int64_t *o = (c & 1) ? off + (np + 1) : off;
            const int64_t a = o[c >> 1], b = o[(c >> 1) + 1];
            cr[2 * (int64_t)c] = a;
            cr[2 * (int64_t)c + 1] = b;
            v = (int32_t)((b - a + kT - 1) / kT);
        }
        int32_t x = v;     // inclusive scan within the wave
        for (int d = 1; d < 64; d <<= 1) {
            const int32_t y = __shfl_up(x, d);
            if (l >= d) x += y;
        }
        if (l == 63) wsum[w] = x;
        __syncthreads();
        int32_t before = 0, total = 0;
        for (int k = 0; k < 16; k++) {
            const int32_t ws = wsum[k];
            before += k < w ? ws : 0;
            total += ws;
        }
        if (c < nc) toff[c] = carry + before + x - v;
        carry += total;
        __syncthreads();   // wsum is rewritten by the next chunk
    }
    if (t == 0) toff[nc] = carry;
}

// per cloud: maximum over its tiles (ties: the lower point index)
__global__ void k_enc_pool(const float *__restrict__ pmax, const int32_t *__restrict__ parg,
                           const int32_t *__restrict__ toff, int nc, float *__restrict__ feat,
                           int32_t *__restrict__ arg)
{
    const int c = blockIdx.x, col = threadIdx.x;
    if (c >= nc) return;
    float best = 0.f;     // an empty cloud has the zero feature
    int32_t barg = -1;
    for (int tl = toff[c]; tl < toff[c + 1]; tl++) {
        float v = pmax[(int64_t)tl * kC3 + col];
        int32_t a = parg[(int64_t)tl * kC3 + col];
        if (a >= 0 && (barg < 0 || v > best)) { best = v; barg = a; }
    }
    feat[(int64_t)c * kC3 + col] = best;
    arg[(int64_t)c * kC3 + col] = barg;
}

__device__ inline void quat_rotation(double w, double x, double y, double z, double R[9])
{
    R[0] = w * w + x * x - y * y - z * z;
    R[1] = 2 * (x * y - w * z);
    R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);
    R[4] = w * w - x * x + y * y - z * z;
    R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);
    R[7] = 2 * (y * z + w * x);
    R[8] = w * w - x * x - y * y + z * z;
}

// T = [R, c_tgt - R c_src]
__device__ inline void pose_about_centroids(const double R[9], const double *cs, const double *ct, double *T)
{
    for (int r = 0; r < 3; r++) {
        for (int cc = 0; cc < 3; cc++) T[r * 4 + cc] = R[r * 3 + cc];
        T[r * 4 + 3] = ct[r] - (R[r * 3] * cs[0] + R[r * 3 + 1] * cs[1] + R[r * 3 + 2] * cs[2]);
    }
    T[12] = T[13] = T[14] = 0.0;
    T[15] = 1.0;
}

// Head per pair (clouds 2p = source, 2p + 1 = target): h = ReLU(W4^T f + b4),
// q = W5^T h + b5, R = rotation of q / |q|, T0 = [R, c_tgt - R c_src].
// A workgroup takes kHeadPairs pairs, so each W4 element it loads feeds
// that many independent sums; every sum runs over its inputs in ascending
// order, one fused multiply-add at a time.
constexpr int kHeadPairs = 4;

__global__ void __launch_bounds__(kH) k_head_forward(const float *__restrict__ feat, const double *__restrict__ cen,
                                                   const float *__restrict__ params, int np,
                                                   float *__restrict__ zbuf, float *__restrict__ qbuf,
                                                   double *__restrict__ out_T)
{
    __shared__ float f[kHeadPairs][2 * kC3];
    __shared__ float h[kHeadPairs][kH];
    __shared__ double qs[kHeadPairs][4];
    __shared__ float sW5[kH * 4];     // W5 staged while h is formed: the q sums then read LDS, not memory
    const int p0 = blockIdx.x * kHeadPairs, j = threadIdx.x;
    const int npb = min(kHeadPairs, np - p0);     // pairs of this workgroup
    if (npb <= 0) return;
    const float *W4 = params + kOffW4, *b4 = params + kOffB4, *W5 = params + kOffW5, *b5 = params + kOffB5;
    for (int e = 0; e < kHeadPairs; e++) {
        const int p = p0 + (e < npb ? e : 0);       // a missing pair repeats the first; nothing of it is written
        f[e][j] = feat[(int64_t)(2 * p) * kC3 + j];
        f[e][kC3 + j] = feat[(int64_t)(2 * p + 1) * kC3 + j];
    }
    for (int x = j; x < kH * 4; x += kH) sW5[x] = W5[x];
    __syncthreads();
    float a[kHeadPairs];
#pragma unroll
    for (int e = 0; e < kHeadPairs; e++) a[e] = b4[j];
    // W4 in batches of kB rows: the next batch's loads are in flight while
    // the current one is summed
    constexpr int kB = 32;
    float wc[kB], wn[kB];
#pragma unroll
    for (int u = 0; u < kB; u++) wc[u] = W4[u * kH + j];
    for (int i0 = 0; i0 < 2 * kC3; i0 += kB) {
        if (i0 + kB < 2 * kC3) {
#pragma unroll
            for (int u = 0; u < kB; u++) wn[u] = W4[(i0 + kB + u) * kH + j];
        }
#pragma unroll
        for (int u = 0; u < kB; u++)
#pragma unroll
            for (int e = 0; e < kHeadPairs; e++) a[e] = __fmaf_rn(f[e][i0 + u], wc[u], a[e]);
#pragma unroll
        for (int u = 0; u < kB; u++) wc[u] = wn[u];
    }
#pragma unroll
    for (int e = 0; e < kHeadPairs; e++) {
        h[e][j] = fmaxf(a[e], 0.f);
        if (e < npb) zbuf[(int64_t)(p0 + e) * kH + j] = a[e];
    }
    __syncthreads();
    if (j < 4 * kHeadPairs) {     // one thread per (pair, quaternion component)
        const int e = j >> 2, o = j & 3;
        float s = b5[o];
#pragma unroll 16
        for (int i = 0; i < kH; i++) s = __fmaf_rn(h[e][i], sW5[i * 4 + o], s);
        qs[e][o] = s;
        if (e < npb) qbuf[(int64_t)(p0 + e) * 4 + o] = s;
    }
    __syncthreads();
    if (j < npb) {
        const int p = p0 + j;
        double q[4] = {qs[j][0], qs[j][1], qs[j][2], qs[j][3]};
        double nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        if (!(nq > 0.0)) { q[0] = 1.0; q[1] = q[2] = q[3] = 0.0; nq = 1.0; }
        double R[9];
        quat_rotation(q[0] / nq, q[1] / nq, q[2] / nq, q[3] / nq, R);
        pose_about_centroids(R, cen + 3 * (2 * p), cen + 3 * (2 * p + 1), out_T + 16 * (int64_t)p);
    }
}

// Per pair: weighted loss w_p |R(q / |q|) - R_label|_F^2 and the backward of
// the head: dq (4), dz4 (256, through the ReLU) and df (512, source then
// target features).
__global__ void __launch_bounds__(kH) k_head_backward(const float *__restrict__ params, int np,
                                                    const float *__restrict__ zbuf, const float *__restrict__ qbuf,
                                                    const double *__restrict__ label_T,
                                                    const float *__restrict__ pair_w, float *__restrict__ loss,
                                                    float *__restrict__ dq_out, float *__restrict__ dz_out,
                                                    float *__restrict__ df_out)
{
    __shared__ float dq[4];
    __shared__ float dz[kH];
    const int p = blockIdx.x, j = threadIdx.x;
    if (p >= np) return;
    if (j == 0) {
        const double wp = pair_w ? (double)pair_w[p] : 1.0;
        double q[4];
        for (int o = 0; o < 4; o++) q[o] = qbuf[(int64_t)p * 4 + o];
        double nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        double g[4] = {0.0, 0.0, 0.0, 0.0}, L = 0.0;
        if (nq > 0.0 && wp != 0.0) {
            double u[4] = {q[0] / nq, q[1] / nq, q[2] / nq, q[3] / nq};
            double R[9], G[9];
            quat_rotation(u[0], u[1], u[2], u[3], R);
            const double *Tl = label_T + 16 * (int64_t)p;
            for (int r = 0; r < 3; r++)
                for (int cc = 0; cc < 3; cc++) {
                    double e = R[r * 3 + cc] - Tl[r * 4 + cc];
                    L += e * e;
                    G[r * 3 + cc] = 2.0 * e;
                }
            // partial derivatives of R in w, x, y, z (row-major 3x3 each)
            const double w = u[0], x = u[1], y = u[2], z = u[3];
            const double D[4][9] = {{2 * w, -2 * z, 2 * y, 2 * z, 2 * w, -2 * x, -2 * y, 2 * x, 2 * w},
                                    {2 * x, 2 * y, 2 * z, 2 * y, -2 * x, -2 * w, 2 * z, 2 * w, -2 * x},
                                    {-2 * y, 2 * x, 2 * w, 2 * x, 2 * y, 2 * z, -2 * w, 2 * z, -2 * y},
                                    {-2 * z, -2 * w, 2 * x, 2 * w, -2 * z, 2 * y, 2 * x, 2 * y, 2 * z}};
            double gu[4], dot = 0.0;
            for (int k = 0; k < 4; k++) {
                gu[k] = 0.0;
                for (int e = 0; e < 9; e++) gu[k] += G[e] * D[k][e];
                dot += gu[k] * u[k];
            }
            // through the normalisation u = q / |q|
            for (int k = 0; k < 4; k++) g[k] = wp * (gu[k] - u[k] * dot) / nq;
            L *= wp;
        }
        for (int o = 0; o < 4; o++) {
            dq[o] = (float)g[o];
            dq_out[(int64_t)p * 4 + o] = (float)g[o];
        }
        loss[p] = (float)L;
    }
    __syncthreads();
    const float *W4 = params + kOffW4, *W5 = params + kOffW5;
    {
        float a = 0.f;
        for (int o = 0; o < 4; o++) a = __fmaf_rn(W5[j * 4 + o], dq[o], a);
        dz[j] = zbuf[(int64_t)p * kH + j] > 0.f ? a : 0.f;
        dz_out[(int64_t)p * kH + j] = dz[j];
    }
    __syncthreads();
    for (int i = j; i < 2 * kC3; i += kH) {
        float a = 0.f;
        for (int k = 0; k < kH; k++) a = __fmaf_rn(W4[i * kH + k], dz[k], a);
        df_out[(int64_t)(2 * p + i / kC3) * kC3 + (i % kC3)] = a;
    }
}

// Head weight gradients, summed over pairs in order: W4 from features x
// dz4 (a workgroup per kGradRows rows of W4, a thread per column, each dz4
// value loaded once for those rows; the features are uniform over the
// workgroup), then b4, W5 from [h, 1] x dq and b5, one thread per weight.
constexpr int kGradRows = 8;
constexpr int kGradW4Blocks = 2 * kC3 / kGradRows;

__global__ void __launch_bounds__(kH) k_head_grads(const float *__restrict__ feat, const float *__restrict__ zbuf,
                                                 const float *__restrict__ dq, const float *__restrict__ dz, int np,
                                                 float *__restrict__ grad)
{
    const int nW5 = kH * 4;
    if ((int)blockIdx.x < kGradW4Blocks) {
        const int i0 = blockIdx.x * kGradRows, j = threadIdx.x;
        const int side = i0 / kC3, c0 = i0 % kC3;     // the rows' cloud (source or target) and channels
        float a[kGradRows];
#pragma unroll
        for (int r = 0; r < kGradRows; r++) a[r] = 0.f;
#pragma unroll 8
        for (int p = 0; p < np; p++) {
            const float d = dz[(int64_t)p * kH + j];
            const float *f = feat + (int64_t)(2 * p + side) * kC3 + c0;
#pragma unroll
            for (int r = 0; r < kGradRows; r++) a[r] = __fmaf_rn(f[r], d, a[r]);
        }
#pragma unroll
        for (int r = 0; r < kGradRows; r++) grad[kOffW4 + (int64_t)(i0 + r) * kH + j] = a[r];
        return;
    }
    const int nrest = kH + nW5 + 4;
    for (int e = (blockIdx.x - kGradW4Blocks) * blockDim.x + threadIdx.x; e < nrest;
         e += (gridDim.x - kGradW4Blocks) * blockDim.x) {
        float a = 0.f;
        if (e < kH) {
            const int jj = e;
            for (int p = 0; p < np; p++) a += dz[(int64_t)p * kH + jj];
            grad[kOffB4 + jj] = a;
        } else if (e < kH + nW5) {
            int k = e - kH, i = k / 4, o = k % 4;
            for (int p = 0; p < np; p++)
                a = __fmaf_rn(fmaxf(zbuf[(int64_t)p * kH + i], 0.f), dq[(int64_t)p * 4 + o], a);
            grad[kOffW5 + k] = a;
        } else {
            int o = e - kH - nW5;
            for (int p = 0; p < np; p++) a += dq[(int64_t)p * 4 + o];
            grad[kOffB5 + o] = a;
        }
    }
}

// Per (cloud c, channel ch) = row e of E = nc * 256: the channel's arg-max
// point, recomputed (bfloat16 inputs and weights as in the forward), and
// the gradient flowing into it.  Writes, k-major with stride E:
//   U1 (4 rows): x, y, z, 1          V1 (64): dz1
//   U2 (65 rows): a1, 1              V2 (128): dz2
//   A2 (128): a2                     G3 (1): dz3 at channel ch
// so that dW1|b1 = U1 V1^T, dW2|b2 = U2 V2^T and dW3[k][ch] = sum over
// clouds of A2[k] G3.  Rows without gradient are all zero.
//
// On the matrix cores, 16 rows per wave (4 waves, 64 rows per workgroup; E
// is a multiple of 64).  Row e = 16 w + lr of the block (lr =
// l % 16) is held by the four lane groups g = l / 16, each with a quarter
// of every channel range, as in the forward's transposed layers:
//   layer 1 (v_mfma_f32_16x16x4_f32) and layer 2 (v_mfma_f32_16x16x32_bf16,
//     W2 in slot order) recompute a1 and a2 exactly as the forward does;
//   dz2[k] = g W3[k][ch] where a2 > 0 (W3 rounded to bfloat16);
//   d1^T = W2 dz2^T on the bfloat16 matrix cores: A = W2 by rows with its
//     columns in slot order (w2q), B = dz2 of this lane's channels, which are
//     that slot order, as hi + lo bfloat16 terms (within 2^-16 of dz2).
__global__ void __launch_bounds__(256) k_enc_backward_mfma(const float *__restrict__ xs, const float *__restrict__ xt,
                                                         const int64_t *__restrict__ cr, int nc,
                                                         const double *__restrict__ cen,
                                                         const float *__restrict__ scale,
                                                         const float *__restrict__ params,
                                                         const __bf16 *__restrict__ w2p, const __bf16 *__restrict__ w2q,
                                                         const __bf16 *__restrict__ w3t, const float *__restrict__ feat,
                                                         const int32_t *__restrict__ arg, const float *__restrict__ df,
                                                         float *__restrict__ U1, float *__restrict__ V1,
                                                         float *__restrict__ U2, float *__restrict__ V2,
                                                         float *__restrict__ A2, float *__restrict__ G3)
{
    const int w = threadIdx.x >> 6, l = __lane_id(), g = l >> 4, lr = l & 15;
    const int64_t E = (int64_t)nc * kC3;
    const int64_t e = (int64_t)blockIdx.x * 64 + 16 * w + lr;
    const int c = (int)(e / kC3), ch = (int)(e % kC3);
    const int32_t r = arg[e];
    const float gv = (r >= 0 && feat[e] > 0.f) ? df[e] : 0.f;
    const bool live = gv != 0.f;
    float x = 0.f, y = 0.f, z = 0.f;
    if (live) norm_point(cloud_xyz(xs, xt, c), cr[2 * c] + r, cen, scale[c], c, x, y, z);
    const float *W1 = params + kOffW1, *b1 = params + kOffB1, *b2 = params + kOffB2;
    // layer 1: lane holds channels 16 t + 4 g + i of its row (t < 4)
    const float bop = g == 0 ? x : (g == 1 ? y : (g == 2 ? z : 1.f));
    float a1v[4][4];
    bf16x8 x1[2];
#pragma unroll
    for (int t = 0; t < kC1 / 16; t++) {
        const int chl = 16 * t + lr;
        const float aop = g < 3 ? W1[g * kC1 + chl] : b1[chl];
        const f32x4 a = __builtin_amdgcn_mfma_f32_16x16x4f32(aop, bop, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const __bf16 h = to_bf16(fmaxf(a[i], 0.f));
            x1[t >> 1][4 * (t & 1) + i] = h;
            a1v[t][i] = (float)h;
        }
    }
    // layer 2: lane holds channels 16 t + 4 g + i (t < 8); then dz2 there
    float dz2[8][4];
#pragma unroll
    for (int t = 0; t < kC2 / 16; t++) {
        f32x4 acc = {b2[16 * t + 4 * g], b2[16 * t + 4 * g + 1], b2[16 * t + 4 * g + 2], b2[16 * t + 4 * g + 3]};
#pragma unroll
        for (int kb = 0; kb < 2; kb++) {
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&w2p[(16 * t + lr) * kC1 + 32 * kb + 8 * g]);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, x1[kb], acc, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int k = 16 * t + 4 * g + i;
            const float a2 = (float)to_bf16(fmaxf(acc[i], 0.f));
            const float d = a2 > 0.f ? gv * (float)w3t[(int64_t)ch * kC2 + k] : 0.f;
            dz2[t][i] = d;
            A2[k * E + e] = live ? a2 : 0.f;
            V2[k * E + e] = d;
        }
    }
    // d1^T[j][row] = sum_k W2[j][k] dz2[k]: k-blocks kb of 32 channels are the
    // lane's tiles (2 kb, 2 kb + 1), i.e. the slot order of w2q
    bf16x8 bh[4], bl[4];
#pragma unroll
    for (int kb = 0; kb < 4; kb++)
#pragma unroll
        for (int jj = 0; jj < 8; jj++) {
            const float v = dz2[2 * kb + (jj >> 2)][jj & 3];
            const __bf16 h = to_bf16(v);
            bh[kb][jj] = h;
            bl[kb][jj] = to_bf16(v - (float)h);
        }
#pragma unroll
    for (int t = 0; t < kC1 / 16; t++) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 4; kb++) {
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&w2q[(16 * t + lr) * kC2 + 32 * kb + 8 * g]);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bh[kb], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bl[kb], acc, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int j = 16 * t + 4 * g + i;
            V1[j * E + e] = a1v[t][i] > 0.f ? acc[i] : 0.f;
            U2[j * E + e] = live ? a1v[t][i] : 0.f;
        }
    }
    if (g == 0) {
        U1[0 * E + e] = x;
        U1[1 * E + e] = y;
        U1[2 * E + e] = z;
        U1[3 * E + e] = live ? 1.f : 0.f;
        U2[kC1 * E + e] = live ? 1.f : 0.f;
        G3[e] = gv;
    }
}

// Partial sums of out[a][b] = sum over rows e of U[a][e] V[b][e], one chunk
// of kChunk rows per workgroup: part[chunk][a * NB + b].
template <int NA, int NB>
__global__ void __launch_bounds__(256) k_outer_partial(const float *__restrict__ U, const float *__restrict__ V,
                                                     int64_t E, float *__restrict__ part)
{
    constexpr int kOut = (NA * NB + 255) / 256;
    constexpr int kS = kChunk + 1;              // padded row stride (bank spread)
    __shared__ float sU[NA * kS];
    __shared__ float sV[NB * kS];
    const int64_t e0 = (int64_t)blockIdx.x * kChunk;
    const int t = threadIdx.x;
    for (int i = t; i < NA * kChunk; i += 256) {
        int a = i / kChunk, r = i % kChunk;
        sU[a * kS + r] = e0 + r < E ? U[a * E + e0 + r] : 0.f;
    }
    for (int i = t; i < NB * kChunk; i += 256) {
        int b = i / kChunk, r = i % kChunk;
        sV[b * kS + r] = e0 + r < E ? V[b * E + e0 + r] : 0.f;
    }
    __syncthreads();
    float acc[kOut];
    for (int o = 0; o < kOut; o++) acc[o] = 0.f;
    for (int r = 0; r < kChunk; r++)
        for (int o = 0; o < kOut; o++) {
            const int idx = t + 256 * o;
            if (idx < NA * NB) acc[o] = __fmaf_rn(sU[(idx / NB) * kS + r], sV[(idx % NB) * kS + r], acc[o]);
        }
    for (int o = 0; o < kOut; o++) {
        const int idx = t + 256 * o;
        if (idx < NA * NB) part[(int64_t)blockIdx.x * (NA * NB) + idx] = acc[o];
    }
}

// Second-layer weight gradients on the bfloat16 matrix cores: partial sums
// of [dW2; db2][a][b] = sum over rows e of U2[a][e] V2[b][e] (a < 65: a1 and
// the constant 1; b < 128: dz2), one chunk of kChunk rows per workgroup,
// part[chunk][a * 128 + b] as k_outer_partial writes them.  U2 holds a1,
// which the forward rounded to bfloat16, and ones: exact in bfloat16.  V2
// (dz2) is float32, so it enters as two bfloat16 terms hi + lo (hi the
// nearest bfloat16, lo that of the remainder; together within 2^-16 of
// dz2), each product exact in float32, accumulated in float32 in a fixed
// order (v_mfma_f32_16x16x32_bf16 over k-steps of 32 rows).  Wave w owns
// output columns 32 w .. 32 w + 31 (two 16-column tiles) and all rows as
// five 16-row tiles (rows 65..79 are zero).  Operand layout as in
// k_enc_forward: lane l supplies A[l % 16][8 g + j] and B[8 g + j][l % 16]
// (g = l / 16, j < 8) and receives C[4 g + i][l % 16].
__global__ void __launch_bounds__(256) k_outer_w2_mfma(const float *__restrict__ U, const float *__restrict__ V,
                                                     int64_t E, float *__restrict__ part)
{
    static_assert(kChunk % 32 == 0 && kC2 == 4 * 32 && kC1 == 64, "tile shapes");
    const int w = threadIdx.x >> 6, l = __lane_id(), g = l >> 4, r = l & 15;
    const int64_t e0 = (int64_t)blockIdx.x * kChunk;
    f32x4 acc[5][2];
#pragma unroll
    for (int mt = 0; mt < 5; mt++)
#pragma unroll
        for (int nt = 0; nt < 2; nt++) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < kChunk; ks += 32) {
        const int64_t eb = e0 + ks + 8 * g;        // this lane's 8 rows of the k-step
        bf16x8 A[5];
#pragma unroll
        for (int mt = 0; mt < 5; mt++) {
            const int a = 16 * mt + r;
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const bool in = eb + j < E;
                const float u = a < kC1 ? (in ? U[(int64_t)a * E + eb + j] : 0.f) : (a == kC1 && in ? 1.f : 0.f);
                A[mt][j] = to_bf16(u);
            }
        }
#pragma unroll
        for (int nt = 0; nt < 2; nt++) {
            const int b = 32 * w + 16 * nt + r;
            bf16x8 hi, lo;
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const float v = eb + j < E ? V[(int64_t)b * E + eb + j] : 0.f;
                const __bf16 h = to_bf16(v);
                hi[j] = h;
                lo[j] = to_bf16(v - (float)h);
            }
#pragma unroll
            for (int mt = 0; mt < 5; mt++) {
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mt], hi, acc[mt][nt], 0, 0, 0);
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mt], lo, acc[mt][nt], 0, 0, 0);
            }
        }
    }
    float *out = part + (int64_t)blockIdx.x * ((kC1 + 1) * kC2);
#pragma unroll
    for (int mt = 0; mt < 5; mt++)
#pragma unroll
        for (int nt = 0; nt < 2; nt++)
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int a = 16 * mt + 4 * g + i, b = 32 * w + 16 * nt + r;
                if (a <= kC1) out[a * kC2 + b] = acc[mt][nt][i];
            }
}

// sum of the chunk partials, in chunk order
__global__ void k_outer_reduce(const float *__restrict__ part, int nchunk, int nout, float *__restrict__ out)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nout; i += gridDim.x * blockDim.x) {
        float a = 0.f;
        // unrolled so the loads go out ahead of the (ordered) additions
#pragma unroll 16
        for (int ch = 0; ch < nchunk; ch++) a += part[(int64_t)ch * nout + i];
        out[i] = a;
    }
}

// third-layer gradients, one thread per weight, summed over clouds in order
__global__ void k_w3_grads(const float *__restrict__ A2, const float *__restrict__ G3, int nc,
                           float *__restrict__ grad)
{
    const int64_t E = (int64_t)nc * kC3;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kC2 * kC3 + kC3; i += gridDim.x * blockDim.x) {
        float a = 0.f;
        if (i < kC2 * kC3) {
            const int k = i / kC3, ch = i % kC3;
#pragma unroll 16
            for (int c = 0; c < nc; c++)
                a = __fmaf_rn(A2[k * E + (int64_t)c * kC3 + ch], G3[(int64_t)c * kC3 + ch], a);
            grad[kOffW3 + i] = a;
        } else {
            const int ch = i - kC2 * kC3;
            for (int c = 0; c < nc; c++) a += G3[(int64_t)c * kC3 + ch];
            grad[kOffB3 + ch] = a;
        }
    }
}

// Adam on every parameter with the gradient of the weighted mean loss
// (the summed gradient divided by the sum of the pair weights).
__global__ void k_adam(float *__restrict__ params, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ grad, const float *__restrict__ pair_w, int np, int step, float lr)
{
    float wsum = 0.f;
    for (int p = 0; p < np; p++) wsum += pair_w ? pair_w[p] : 1.f;
    if (!(wsum > 0.f)) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kParams; i += gridDim.x * blockDim.x) {
        float g = grad[i] / wsum;
        float mi = b1 * m[i] + (1.f - b1) * g;
        float vi = b2 * v[i] + (1.f - b2) * g * g;
        m[i] = mi;
        v[i] = vi;
        params[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// Multi-start poses for the listed pairs: start j = 0 is the identity
// rotation, start j >= 1 the rotation by 60 degrees about Fibonacci-sphere
// axis j - 1 of 7 (height 1 - (2i + 1) / 7, azimuth i times the golden
// angle), each about the source centroid onto the target centroid.
__global__ void k_start_poses(const double *__restrict__ cen, const int32_t *__restrict__ sel, int nsel,
                              double *__restrict__ out_T)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsel * kStarts) return;
    const int p = sel[i / kStarts], j = i % kStarts;
    double R[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    if (j > 0) {
        const int a = j - 1;
        const double golden = M_PI * (3.0 - sqrt(5.0));
        const double zc = 1.0 - (2.0 * a + 1.0) / (kStarts - 1);
        const double rc = sqrt(fmax(0.0, 1.0 - zc * zc));
        const double ax[3] = {rc * cos(a * golden), rc * sin(a * golden), zc};
        const double th = M_PI / 3.0, s = sin(th), c1 = 1.0 - cos(th);
        // Rodrigues: I + sin(th) K + (1 - cos(th)) K^2, K the cross-product matrix
        const double K[9] = {0, -ax[2], ax[1], ax[2], 0, -ax[0], -ax[1], ax[0], 0};
        for (int r = 0; r < 3; r++)
            for (int cc = 0; cc < 3; cc++) {
                double k2 = 0.0;
                for (int m = 0; m < 3; m++) k2 += K[r * 3 + m] * K[m * 3 + cc];
                R[r * 3 + cc] = (r == cc ? 1.0 : 0.0) + s * K[r * 3 + cc] + c1 * k2;
            }
    }
    pose_about_centroids(R, cen + 3 * (2 * p), cen + 3 * (2 * p + 1), out_T + 16 * (int64_t)i);
}

// Best start per listed pair: the first start, replaced by a later one that
// has inliers and either the best so far has none or its RMS is lower.
__global__ void k_select_start(const double *__restrict__ T_all, const pc_icp_stats *__restrict__ st_all,
                               const int32_t *__restrict__ sel, int nsel, double *__restrict__ out_T,
                               pc_icp_stats *__restrict__ out_stats, int32_t *__restrict__ out_start)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsel) return;
    const pc_icp_stats *s = st_all + (int64_t)i * kStarts;
    int best = 0;
    for (int j = 1; j < kStarts; j++)
        if (s[j].inliers > 0 && (s[best].inliers == 0 || s[j].rms < s[best].rms)) best = j;
    const int p = sel[i];
    for (int k = 0; k < 16; k++) out_T[16 * (int64_t)p + k] = T_all[16 * ((int64_t)i * kStarts + best) + k];
    if (out_stats) out_stats[p] = s[best];
    if (out_start) out_start[p] = best;
}

// rows of 3 floats: segment q copies seg[3q + 2] rows from row seg[3q + 1]
// of `in` to row seg[3q] of `out`
__global__ void k_gather_rows3(const float *__restrict__ in, float *__restrict__ out,
                               const int64_t *__restrict__ seg, int nseg)
{
    for (int q = blockIdx.x; q < nseg; q += gridDim.x) {
        const int64_t d = 3 * seg[3 * q], s = 3 * seg[3 * q + 1], n = 3 * seg[3 * q + 2];
        for (int64_t k = threadIdx.x; k < n; k += blockDim.x) out[d + k] = in[s + k];
    }
}

__global__ void k_fill_i32(int32_t *__restrict__ p, int n, int32_t v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

int pose_net_tiles(int64_t n_cloud) { return (int)((n_cloud + kT - 1) / kT); }

void pose_net_carve(Carver &c, int np, int ntile, bool train, PoseNetStore &s)
{
    const int np1 = np > 0 ? np : 1, nc = 2 * np1, nt1 = ntile > 0 ? ntile : 1;
    const int64_t E = (int64_t)nc * kC3;
    s = PoseNetStore{};
    s.np = np1;
    s.nc = nc;
    s.ntile = ntile;
    s.offs = c.take<int64_t>((size_t)2 * (np1 + 1));
    s.cr = c.take<int64_t>((size_t)2 * nc);
    s.toff = c.take<int32_t>(nc + 1);
    s.cen = c.take<double>((size_t)nc * 3);
    s.scale = c.take<float>(nc);
    s.w3t = c.take<__bf16>(kC2 * kC3);
    s.w3p = c.take<__bf16>(kC2 * kC3);
    s.w2p = c.take<__bf16>(kC1 * kC2);
    s.w2q = c.take<__bf16>(kC1 * kC2);
    s.pmax = c.take<float>((size_t)nt1 * kC3);
    s.parg = c.take<int32_t>((size_t)nt1 * kC3);
    s.feat = c.take<float>((size_t)nc * kC3);
    s.arg = c.take<int32_t>((size_t)nc * kC3);
    s.z4 = c.take<float>((size_t)np1 * kH);
    s.q = c.take<float>((size_t)np1 * 4);
    s.T = c.take<double>((size_t)np1 * 16);
    if (!train) return;
    s.nchunk = (int)((E + kChunk - 1) / kChunk);
    s.grad = c.take<float>(kParams);
    s.loss = c.take<float>(np1);
    s.dq = c.take<float>((size_t)np1 * 4);
    s.dz = c.take<float>((size_t)np1 * kH);
    s.df = c.take<float>((size_t)nc * kC3);
    s.U1 = c.take<float>((size_t)4 * E);
    s.V1 = c.take<float>((size_t)kC1 * E);
    s.U2 = c.take<float>((size_t)(kC1 + 1) * E);
    s.V2 = c.take<float>((size_t)kC2 * E);
    s.A2 = c.take<float>((size_t)kC2 * E);
    s.G3 = c.take<float>((size_t)E);
    s.part = c.take<float>((size_t)s.nchunk * (kC1 + 1) * kC2);
}

hipError_t pose_net_layout(PoseNetStore &s, hipStream_t st)
{
    k_pose_layout<<<1, 1024, 0, st>>>(s.offs, s.np, s.cr, s.toff);
    return hipGetLastError();
}

hipError_t pose_net_stats(PoseNetStore &s, const float *xs, const float *xt, hipStream_t st)
{
    k_norm_stats<<<s.nc, 256, 0, st>>>(xs, xt, s.cr, s.nc, s.cen, s.scale);
    return hipGetLastError();
}

namespace {

// enc_slot >= 0: the kernel timer slot recorded around the encoder kernel
hipError_t forward_impl(PoseNetStore &s, const float *params, const float *xs, const float *xt, double *out_T,
                        bool want_arg, int enc_slot, hipStream_t st)
{
    k_norm_stats<<<s.nc, 256, 0, st>>>(xs, xt, s.cr, s.nc, s.cen, s.scale);
    k_weights_bf16<<<64, 256, 0, st>>>(params, s.w3t, s.w3p, s.w2p, s.w2q);
    if (s.ntile > 0) {
        // one persistent workgroup per compute unit (LDS holds one), or fewer
        const int grid = s.ntile < 256 ? s.ntile : 256;
        if (enc_slot >= 0) timer_slot_begin(enc_slot, st);
        if (want_arg)
            k_enc_forward<true><<<grid, kEncThreads, 0, st>>>(xs, xt, s.cr, s.toff, s.nc, s.ntile, s.cen, s.scale,
                                                              params, s.w2p, s.w3p, s.pmax, s.parg);
        else
            k_enc_forward<false><<<grid, kEncThreads, 0, st>>>(xs, xt, s.cr, s.toff, s.nc, s.ntile, s.cen, s.scale,
                                                               params, s.w2p, s.w3p, s.pmax, s.parg);
        if (enc_slot >= 0) timer_slot_end(enc_slot, st);
    }
    k_enc_pool<<<s.nc, kC3, 0, st>>>(s.pmax, s.parg, s.toff, s.nc, s.feat, s.arg);
    k_head_forward<<<(s.np + kHeadPairs - 1) / kHeadPairs, kH, 0, st>>>(s.feat, s.cen, params, s.np, s.z4, s.q,
                                                                        out_T ? out_T : s.T);
    return hipGetLastError();
}

}  // namespace

hipError_t pose_net_forward(PoseNetStore &s, const float *params, const float *xs, const float *xt, double *out_T,
                            hipStream_t st, int enc_slot)
{
    return forward_impl(s, params, xs, xt, out_T, false, enc_slot, st);
}

hipError_t pose_net_train(PoseNetStore &s, float *params, float *adam_m, float *adam_v, int step, float lr,
                          const float *xs, const float *xt, const double *label_T, const float *pair_w,
                          float *out_loss, hipStream_t st)
{
    // timer slots (pc_set_kernel_timer): 0 forward, 1 backward, 2 the
    // second-layer weight gradients on the matrix cores
    timer_slot_begin(0, st);
    hipError_t e = forward_impl(s, params, xs, xt, nullptr, true, -1, st);
    timer_slot_end(0, st);
    if (e != hipSuccess) return e;
    const int64_t E = (int64_t)s.nc * kC3;
    timer_slot_begin(1, st);
    k_head_backward<<<s.np, kH, 0, st>>>(params, s.np, s.z4, s.q, label_T, pair_w, out_loss ? out_loss : s.loss,
                                        s.dq, s.dz, s.df);
    k_head_grads<<<kGradW4Blocks + (kH + kH * 4 + 4 + kH - 1) / kH, kH, 0, st>>>(s.feat, s.z4, s.dq, s.dz, s.np,
                                                                              s.grad);
    k_enc_backward_mfma<<<(int)(E / 64), 256, 0, st>>>(xs, xt, s.cr, s.nc, s.cen, s.scale, params, s.w2p, s.w2q,
                                                       s.w3t, s.feat, s.arg, s.df, s.U1, s.V1, s.U2, s.V2, s.A2,
                                                       s.G3);
    k_w3_grads<<<128, 256, 0, st>>>(s.A2, s.G3, s.nc, s.grad);
    k_outer_partial<4, kC1><<<s.nchunk, 256, 0, st>>>(s.U1, s.V1, E, s.part);
    k_outer_reduce<<<1, 256, 0, st>>>(s.part, s.nchunk, 4 * kC1, s.grad + kOffW1);
    timer_slot_begin(2, st);
    k_outer_w2_mfma<<<s.nchunk, 256, 0, st>>>(s.U2, s.V2, E, s.part);
    timer_slot_end(2, st);
    k_outer_reduce<<<(((kC1 + 1) * kC2) + 255) / 256, 256, 0, st>>>(s.part, s.nchunk, (kC1 + 1) * kC2,
                                                                      s.grad + kOffW2);
    timer_slot_end(1, st);
    if (lr > 0.f) k_adam<<<256, 256, 0, st>>>(params, adam_m, adam_v, s.grad, pair_w, s.np, step, lr);
    return hipGetLastError();
}

hipError_t multi_start_poses(const double *cen, const int32_t *sel, int nsel, double *out_T, hipStream_t st)
{
    const int n = nsel * kStarts;
    if (n > 0) k_start_poses<<<(n + 63) / 64, 64, 0, st>>>(cen, sel, nsel, out_T);
    return hipGetLastError();
}

hipError_t multi_start_select(const double *T_all, const pc_icp_stats *st_all, const int32_t *sel, int nsel,
                              double *out_T, pc_icp_stats *out_stats, int32_t *out_start, hipStream_t st)
{
    if (nsel > 0)
        k_select_start<<<(nsel + 63) / 64, 64, 0, st>>>(T_all, st_all, sel, nsel, out_T, out_stats, out_start);
    return hipGetLastError();
}

hipError_t gather_rows3(const float *in, float *out, const int64_t *seg, int nseg, hipStream_t st)
{
    if (nseg > 0) k_gather_rows3<<<nseg < 4096 ? nseg : 4096, 256, 0, st>>>(in, out, seg, nseg);
    return hipGetLastError();
}

hipError_t fill_i32(int32_t *p, int n, int32_t v, hipStream_t st)
{
    if (n > 0) k_fill_i32<<<(n + 255) / 256, 256, 0, st>>>(p, n, v);
    return hipGetLastError();
}

}  // namespace pcg
