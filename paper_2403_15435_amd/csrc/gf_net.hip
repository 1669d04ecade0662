// Learned refinement tagger on gfx950: patch features, and a small
// convolutional network (three 3x3 convolutions, mean pooling, a fully
// connected layer) whose convolutions, forward and backward, are implicit
// matrix products on the BF16 matrix cores with FP32 accumulation.
//
// Rounding points (bfloat16, round to nearest even): input features, the
// three conv weight tensors, the post-ReLU activations of layers 1 and 2, and
// the three pre-activation gradients that enter the products.  Biases,
// layer-3 activations, pooling, the fully connected layer, the loss and all
// sums are FP32.  One workgroup per sample holds all its activations in LDS.
#include "gf_net.h"

namespace gfnet {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t to_bf16(float x)
{
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);   // NaN stays NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// One 16 x 16 output tile: acc += A (16 x K) B (K x 16), K a multiple of 16,
// on gfx950's 16x16x32 bf16 matrix instruction, with one 16x16x16 step for
// a 16-wide remainder.  16x16x32: lane l supplies A(l % 16, k0 + 8 (l / 16) + j)
// and B(k0 + 8 (l / 16) + j, l % 16) for j < 8; 16x16x16: the same with 4
// values from k0 + 4 (l / 16).  Either way lane l holds C(4 (l / 16) + r, l % 16)
// for r < 4.
template <class FA, class FB>
__device__ __forceinline__ f32x4 mma_tile(int K, FA fa, FB fb, f32x4 acc)
{
    const int lane = threadIdx.x & 63;
    const int i = lane & 15, g = lane >> 4;
    int k0 = 0;
    for (; k0 + 32 <= K; k0 += 32) {
        bf16x8 av, bv;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            av[j] = __builtin_bit_cast(__bf16, (uint16_t)fa(i, k0 + 8 * g + j));
            bv[j] = __builtin_bit_cast(__bf16, (uint16_t)fb(k0 + 8 * g + j, i));
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
    }
    if (k0 < K) {
        bf16x4 av, bv;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            av[j] = (short)fa(i, k0 + 4 * g + j);
            bv[j] = (short)fb(k0 + 4 * g + j, i);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
    }
    return acc;
}

constexpr int NT = 256, NWV = NT / 64;

struct NetSmem {
    uint16_t X0[FEAT];            // [24 * 24][4]
    uint16_t W1[576], W2[4608], W3[9216];   // [co][tap * cin + ci]
    uint16_t A1[24 * 24 * 16];    // post-ReLU, [p][c]
    uint16_t A2[12 * 12 * 32];
    float Y3[6 * 6 * 32];         // pre-activation of layer 3
    uint16_t dY3[6 * 6 * 32];
    uint16_t dY2[12 * 12 * 32];
    union {
        uint16_t dY1[24 * 24 * 16];
        float dY2f[12 * 12 * 32];   // unrounded layer-2 gradient, for its bias sum
    };
    float P[32], dP[32], Z[4], dZ[4];
    float red[NWV][16];
};

// zero padding of 1 around an h x w image: (y, x) inside?
__device__ __forceinline__ bool inside(int y, int x, int h, int w) { return y >= 0 && y < h && x >= 0 && x < w; }

template <bool TRAIN>
__global__ void __launch_bounds__(NT) net_kernel(const NetArgs a)
{
    __shared__ NetSmem S;
    const int s = blockIdx.x, tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int lrow = 4 * (lane >> 4), lcol = lane & 15;
    for (int i = tid; i < FEAT; i += NT)
        S.X0[i] = a.x ? to_bf16(a.x[(int64_t)s * FEAT + i]) : a.xb[(int64_t)s * FEAT + i];
    for (int i = tid; i < 576; i += NT) S.W1[i] = a.wb[OFF_W1 + i];
    for (int i = tid; i < 4608; i += NT) S.W2[i] = a.wb[OFF_W2 + i];
    for (int i = tid; i < 9216; i += NT) S.W3[i] = a.wb[OFF_W3 + i];
    __syncthreads();
    const float *w = a.w;
    // conv1, stride 1: 576 pixels x 16 channels, K = 9 taps x 4 (36, padded to 48)
    for (int t = wv; t < 36; t += NWV) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mma_tile(48,
            [&](int i, int k) -> uint16_t {
                if (k >= 36) return 0;
                const int p = t * 16 + i, y = p / 24, x = p % 24, tap = k >> 2, ci = k & 3;
                const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
                return inside(yy, xx, 24, 24) ? S.X0[(yy * 24 + xx) * 4 + ci] : (uint16_t)0;
            },
            [&](int k, int j) -> uint16_t { return k < 36 ? S.W1[j * 36 + k] : (uint16_t)0; }, acc);
        for (int r = 0; r < 4; ++r) {
            const int p = t * 16 + lrow + r, co = lcol;
            S.A1[p * 16 + co] = to_bf16(fmaxf(acc[r] + w[OFF_B1 + co], 0.f));
        }
    }
    __syncthreads();
    // conv2, stride 2: 144 pixels x 32 channels, K = 9 x 16
    for (int t = wv; t < 18; t += NWV) {
        const int mt = t >> 1, nt = t & 1;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mma_tile(144,
            [&](int i, int k) -> uint16_t {
                const int p = mt * 16 + i, oy = p / 12, ox = p % 12, tap = k >> 4, ci = k & 15;
                const int yy = 2 * oy + tap / 3 - 1, xx = 2 * ox + tap % 3 - 1;
                return inside(yy, xx, 24, 24) ? S.A1[(yy * 24 + xx) * 16 + ci] : (uint16_t)0;
            },
            [&](int k, int j) -> uint16_t { return S.W2[(nt * 16 + j) * 144 + k]; }, acc);
        for (int r = 0; r < 4; ++r) {
            const int p = mt * 16 + lrow + r, co = nt * 16 + lcol;
            S.A2[p * 32 + co] = to_bf16(fmaxf(acc[r] + w[OFF_B2 + co], 0.f));
        }
    }
    __syncthreads();
    // conv3, stride 2: 36 pixels (padded to 48) x 32 channels, K = 9 x 32
    for (int t = wv; t < 6; t += NWV) {
        const int mt = t >> 1, nt = t & 1;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mma_tile(288,
            [&](int i, int k) -> uint16_t {
                const int p = mt * 16 + i;
                if (p >= 36) return 0;
                const int oy = p / 6, ox = p % 6, tap = k >> 5, ci = k & 31;
                const int yy = 2 * oy + tap / 3 - 1, xx = 2 * ox + tap % 3 - 1;
                return inside(yy, xx, 12, 12) ? S.A2[(yy * 12 + xx) * 32 + ci] : (uint16_t)0;
            },
            [&](int k, int j) -> uint16_t { return S.W3[(nt * 16 + j) * 288 + k]; }, acc);
        for (int r = 0; r < 4; ++r) {
            const int p = mt * 16 + lrow + r, co = nt * 16 + lcol;
            if (p < 36) S.Y3[p * 32 + co] = acc[r] + w[OFF_B3 + co];
        }
    }
    __syncthreads();
    // mean pooling and the fully connected layer (FP32)
    if (tid < 32) {
        float sum = 0.f;
        for (int p = 0; p < 36; ++p) sum += fmaxf(S.Y3[p * 32 + tid], 0.f);
        S.P[tid] = sum / 36.f;
    }
    __syncthreads();
    if (tid < 3) {
        float z = w[OFF_BF + tid];
        for (int c = 0; c < 32; ++c) z += S.P[c] * w[OFF_WF + tid * 32 + c];
        S.Z[tid] = z;
        a.logits[(int64_t)s * 3 + tid] = z;
    }
    if (!TRAIN) return;
    __syncthreads();
    // weighted cross-entropy and its gradient in the logits
    if (tid == 0) {
        const float zm = fmaxf(fmaxf(S.Z[0], S.Z[1]), S.Z[2]);
        float e[3], es = 0.f;
        for (int j = 0; j < 3; ++j) { e[j] = expf(S.Z[j] - zm); es += e[j]; }
        // a label outside 0..2 (possible only for batches given in device
        // memory) weighs 0; so does every sample of a batch whose weights sum to 0
        const int yl = a.y[s];
        const bool valid = yl >= 0 && yl <= 2;
        const int y = valid ? yl : 1;
        const float wt = a.wtot_dev ? *a.wtot_dev : a.wtot;
        const float wy = valid && wt > 0.f ? a.cw[y] : 0.f;
        const float den = wt > 0.f ? wt : 1.f;
        a.loss_i[s] = wy * -logf(e[y] / es) / den;
        for (int j = 0; j < 3; ++j) S.dZ[j] = (wy / den) * (e[j] / es - (j == y ? 1.f : 0.f));
    }
    __syncthreads();
    float *g = a.part + (int64_t)s * N_PARAMS;
    if (tid < 96) g[OFF_WF + tid] = S.dZ[tid / 32] * S.P[tid % 32];
    if (tid < 3) g[OFF_BF + tid] = S.dZ[tid];
    if (tid < 32) {
        float dp = 0.f;
        for (int j = 0; j < 3; ++j) dp += S.dZ[j] * w[OFF_WF + j * 32 + tid];
        S.dP[tid] = dp;
    }
    __syncthreads();
    // layer 3: dY3 = dP / 36 where Y3 > 0
    for (int i = tid; i < 36 * 32; i += NT) S.dY3[i] = to_bf16(S.Y3[i] > 0.f ? S.dP[i & 31] / 36.f : 0.f);
    if (tid < 32) {
        float sb = 0.f;
        for (int p = 0; p < 36; ++p) sb += S.Y3[p * 32 + tid] > 0.f ? S.dP[tid] / 36.f : 0.f;
        g[OFF_B3 + tid] = sb;
    }
    __syncthreads();
    // dW3[co][k] = sum over the 36 pixels of im2col(A2)[p][k] dY3[p][co]
    for (int t = wv; t < 36; t += NWV) {
        const int kt = t >> 1, nt = t & 1;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mma_tile(48,
            [&](int i, int kk) -> uint16_t {
                const int k = kt * 16 + i, p = kk;
                if (p >= 36) return 0;
                const int oy = p / 6, ox = p % 6, tap = k >> 5, ci = k & 31;
                const int yy = 2 * oy + tap / 3 - 1, xx = 2 * ox + tap % 3 - 1;
                return inside(yy, xx, 12, 12) ? S.A2[(yy * 12 + xx) * 32 + ci] : (uint16_t)0;
            },
            [&](int kk, int j) -> uint16_t { return kk < 36 ? S.dY3[kk * 32 + nt * 16 + j] : (uint16_t)0; }, acc);
        for (int r = 0; r < 4; ++r) g[OFF_W3 + (nt * 16 + lcol) * 288 + kt * 16 + lrow + r] = acc[r];
    }
    // dA2[q][ci] = sum over taps and co of dY3[output pixel reading q through the tap][co] W3[co][tap][ci]
    for (int t = wv; t < 18; t += NWV) {
        const int mt = t >> 1, nt = t & 1;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mma_tile(288,
            [&](int i, int kk) -> uint16_t {
                const int q = mt * 16 + i, qy = q / 12, qx = q % 12, tap = kk >> 5, co = kk & 31;
                const int ty = qy + 1 - tap / 3, tx = qx + 1 - tap % 3;
                if (ty < 0 || tx < 0 || (ty & 1) || (tx & 1) || ty >= 12 || tx >= 12) return 0;
                return S.dY3[((ty >> 1) * 6 + (tx >> 1)) * 32 + co];
            },
            [&](int kk, int j) -> uint16_t { return S.W3[(kk & 31) * 288 + (kk >> 5) * 32 + nt * 16 + j]; }, acc);
        for (int r = 0; r < 4; ++r) {
            const int q = mt * 16 + lrow + r, ci = nt * 16 + lcol;
            const float v = from_bf16(S.A2[q * 32 + ci]) > 0.f ? acc[r] : 0.f;
            S.dY2f[q * 32 + ci] = v;
            S.dY2[q * 32 + ci] = to_bf16(v);
        }
    }
    __syncthreads();
    if (tid < 32) {
        float sb = 0.f;
        for (int q = 0; q < 144; ++q) sb += S.dY2f[q * 32 + tid];
        g[OFF_B2 + tid] = sb;
    }
    // dW2[co][k] = sum over the 144 conv2 outputs of im2col(A1)[p][k] dY2[p][co]
    for (int t = wv; t < 18; t += NWV) {
        const int kt = t >> 1, nt = t & 1;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mma_tile(144,
            [&](int i, int kk) -> uint16_t {
                const int k = kt * 16 + i, p = kk, oy = p / 12, ox = p % 12, tap = k >> 4, ci = k & 15;
                const int yy = 2 * oy + tap / 3 - 1, xx = 2 * ox + tap % 3 - 1;
                return inside(yy, xx, 24, 24) ? S.A1[(yy * 24 + xx) * 16 + ci] : (uint16_t)0;
            },
            [&](int kk, int j) -> uint16_t { return S.dY2[kk * 32 + nt * 16 + j]; }, acc);
        for (int r = 0; r < 4; ++r) g[OFF_W2 + (nt * 16 + lcol) * 144 + kt * 16 + lrow + r] = acc[r];
    }
    __syncthreads();   // the bias sum above read dY2f, which dY1 overwrites
    // dA1[q][ci] = sum over taps and co of dY2[output pixel reading q][co] W2[co][tap][ci]
    float b1p = 0.f;   // this lane's share of the layer-1 bias gradient (channel lcol)
    for (int t = wv; t < 36; t += NWV) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mma_tile(288,
            [&](int i, int kk) -> uint16_t {
                const int q = t * 16 + i, qy = q / 24, qx = q % 24, tap = kk >> 5, co = kk & 31;
                const int ty = qy + 1 - tap / 3, tx = qx + 1 - tap % 3;
                if (ty < 0 || tx < 0 || (ty & 1) || (tx & 1) || ty >= 24 || tx >= 24) return 0;
                return S.dY2[((ty >> 1) * 12 + (tx >> 1)) * 32 + co];
            },
            [&](int kk, int j) -> uint16_t { return S.W2[(kk & 31) * 144 + (kk >> 5) * 16 + j]; }, acc);
        for (int r = 0; r < 4; ++r) {
            const int q = t * 16 + lrow + r, ci = lcol;
            const float v = from_bf16(S.A1[q * 16 + ci]) > 0.f ? acc[r] : 0.f;
            S.dY1[q * 16 + ci] = to_bf16(v);
            b1p += v;
        }
    }
    // layer-1 bias: lanes l, l+16, l+32, l+48 share a channel; then waves in order
    b1p += __shfl_xor(b1p, 16);
    b1p += __shfl_xor(b1p, 32);
    if (lane < 16) S.red[wv][lane] = b1p;
    __syncthreads();
    if (tid < 16) {
        float sb = 0.f;
        for (int k = 0; k < NWV; ++k) sb += S.red[k][tid];
        g[OFF_B1 + tid] = sb;
    }
    // dW1[co][k] = sum over the 576 pixels of im2col(X0)[q][k] dY1[q][co]
    for (int t = wv; t < 3; t += NWV) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mma_tile(576,
            [&](int i, int kk) -> uint16_t {
                const int k = t * 16 + i, q = kk;
                if (k >= 36) return 0;
                const int qy = q / 24, qx = q % 24, tap = k >> 2, ci = k & 3;
                const int yy = qy + tap / 3 - 1, xx = qx + tap % 3 - 1;
                return inside(yy, xx, 24, 24) ? S.X0[(yy * 24 + xx) * 4 + ci] : (uint16_t)0;
            },
            [&](int kk, int j) -> uint16_t { return S.dY1[kk * 16 + j]; }, acc);
        for (int r = 0; r < 4; ++r) {
            const int k = t * 16 + lrow + r;
            if (k < 36) g[OFF_W1 + lcol * 36 + k] = acc[r];
        }
    }
}

// grad[i] = sum over samples in order of part[s][i]
__global__ void __launch_bounds__(256) reduce_kernel(const float *part, int n, float *grad)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= N_PARAMS) return;
    float sum = 0.f;
    for (int s = 0; s < n; ++s) sum += part[(int64_t)s * N_PARAMS + i];
    grad[i] = sum;
}

// Adam (beta1 0.9, beta2 0.999, eps 1e-8); bc1 = 1 - beta1^t, bc2 = 1 - beta2^t
__global__ void __launch_bounds__(256) adam_kernel(float *w, float *m, float *v, uint16_t *wb, const float *g, float lr,
                                                   float bc1, float bc2)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= N_PARAMS) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + 1e-8f);
    w[i] = wi;
    wb[i] = to_bf16(wi);
}

__global__ void __launch_bounds__(256) to_bf16_kernel(const float *w, uint16_t *wb, int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) wb[i] = to_bf16(w[i]);
}

// ---------------------------------------------------------------------------
// features
// ---------------------------------------------------------------------------

// Finest image of one scenario: pixel (px, py) is the mean over its square
// (m/8 finest-level cells on a side) of the leaf fields h, hu, hv, b.  The
// covering leaf is found by walking the per-level slot maps from the finest
// level up.
template <typename RS>
__global__ void __launch_bounds__(256) image_kernel(const RS *q, const RS *b, int64_t cap, int m, const int32_t *map,
                                                    const FeatLevel *lv, int Lf, int nx, int ny, float *img)
{
    const int px = blockIdx.x * 256 + threadIdx.x, py = blockIdx.y;
    if (px >= nx || py >= ny) return;
    const int PIf = px >> 3, PJf = py >> 3;
    int L = Lf, slot = -1;
    for (; L >= 0; --L) {
        const int sh = Lf - L;
        const int s = map[lv[L].map_off + (int64_t)(PJf >> sh) * lv[L].map_w + (PIf >> sh)];
        if (s >= 0) { slot = s; break; }
    }
    const int64_t plane = (int64_t)nx * ny, o = (int64_t)py * nx + px;
    if (slot < 0) {
        for (int c = 0; c < 4; ++c) img[c * plane + o] = 0.f;
        return;
    }
    const int sh = Lf - L, cpp = m / 8;
    const int n = (cpp >> sh) > 0 ? (cpp >> sh) : 1;      // leaf cells per pixel side
    const int gx = (px * cpp) >> sh, gy = (py * cpp) >> sh;   // first covered cell, global at level L
    const int lx = gx - (PIf >> sh) * m, ly = gy - (PJf >> sh) * m;
    const int64_t MM = (int64_t)m * m, fs = cap * MM, base = (int64_t)slot * MM;
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            const int64_t c = base + (int64_t)(ly + j) * m + (lx + i);
            acc[0] += (float)q[c];
            acc[1] += (float)q[fs + c];
            acc[2] += (float)q[2 * fs + c];
            acc[3] += (float)b[c];
        }
    const float inv = 1.f / (float)(n * n);
    for (int c = 0; c < 4; ++c) img[c * plane + o] = acc[c] * inv;
}

// coarser image: each pixel the mean of its 2 x 2 finer pixels
__global__ void __launch_bounds__(256) pyramid_kernel(const float *fine, int fnx, int fny, float *coarse, int cnx,
                                                      int cny)
{
    const int px = blockIdx.x * 256 + threadIdx.x, py = blockIdx.y;
    if (px >= cnx || py >= cny) return;
    const int64_t fp = (int64_t)fnx * fny, cp = (int64_t)cnx * cny;
    for (int c = 0; c < 4; ++c) {
        const float *f = fine + c * fp;
        const float a00 = f[(int64_t)(2 * py) * fnx + 2 * px], a01 = f[(int64_t)(2 * py) * fnx + 2 * px + 1];
        const float a10 = f[(int64_t)(2 * py + 1) * fnx + 2 * px], a11 = f[(int64_t)(2 * py + 1) * fnx + 2 * px + 1];
        coarse[c * cp + (int64_t)py * cnx + px] = 0.25f * ((a00 + a11) + (a01 + a10));
    }
}

// Feature tile of a leaf: the 24 x 24 pixels of its level's image around it
// (3 x 3 patch squares), zero outside the domain; bed relative to the leaf's
// own mean bed; channels scaled by 1, 1/10, 1/10, 1/10.
__global__ void __launch_bounds__(256) tile_kernel(const float *img, const FeatLevel *lv, const int32_t *leaf_lij,
                                                   float *featf, uint16_t *featb)
{
    __shared__ float red[4];
    const int k = blockIdx.x, tid = threadIdx.x;
    const int l = leaf_lij[3 * k], PI = leaf_lij[3 * k + 1], PJ = leaf_lij[3 * k + 2];
    const FeatLevel L = lv[l];
    const float *im = img + L.img_off;
    const int64_t plane = (int64_t)L.nx * L.ny;
    // mean bed of the leaf: its own 8 x 8 pixels
    float bs = 0.f;
    if (tid < 64) bs = im[3 * plane + (int64_t)(8 * PJ + (tid >> 3)) * L.nx + 8 * PI + (tid & 7)];
    for (int off = 32; off > 0; off >>= 1) bs += __shfl_xor(bs, off);
    if (tid == 0) red[0] = bs / 64.f;
    __syncthreads();
    const float bleaf = red[0];
    const float scale[4] = {1.f, 0.1f, 0.1f, 0.1f};
    for (int e = tid; e < TILE * TILE; e += 256) {
        const int y = e / TILE, x = e % TILE;
        const int gy = 8 * PJ - 8 + y, gx = 8 * PI - 8 + x;
        const bool in = gy >= 0 && gy < L.ny && gx >= 0 && gx < L.nx;
        for (int c = 0; c < 4; ++c) {
            float v = 0.f;
            if (in) {
                v = im[c * plane + (int64_t)gy * L.nx + gx];
                if (c == 3) v -= bleaf;
                v *= scale[c];
            }
            featf[(int64_t)k * FEAT + e * 4 + c] = v;
            featb[(int64_t)k * FEAT + e * 4 + c] = to_bf16(v);
        }
    }
}

}  // namespace gfnet

using namespace gfnet;

hipError_t gfnet_launch_forward(const NetArgs &a, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(net_kernel<false>, dim3(a.n), dim3(NT), 0, s, a);
    return hipGetLastError();
}

hipError_t gfnet_launch_train(const NetArgs &a, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(net_kernel<true>, dim3(a.n), dim3(NT), 0, s, a);
    return hipGetLastError();
}

// one workgroup: per-lane sums in label order, then a fixed tree
__global__ void __launch_bounds__(256) weight_sum_kernel(const int8_t *y, int n, float c0, float c1, float c2,
                                                         float *wtot)
{
    __shared__ float part[256];
    const int tid = threadIdx.x;
    float acc = 0.f;
    for (int i = tid; i < n; i += 256) {
        const int l = y[i];
        acc += l == 0 ? c0 : (l == 1 ? c1 : (l == 2 ? c2 : 0.f));
    }
    part[tid] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) part[tid] += part[tid + w];
        __syncthreads();
    }
    if (tid == 0) *wtot = part[0];
}

hipError_t gfnet_launch_reduce(const float *part, int n, float *grad, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_kernel, dim3((N_PARAMS + 255) / 256), dim3(256), 0, s, part, n, grad);
    return hipGetLastError();
}

hipError_t gfnet_launch_weight_sum(const int8_t *y, int n, float c0, float c1, float c2, float *wtot, hipStream_t s)
{
    hipLaunchKernelGGL(weight_sum_kernel, dim3(1), dim3(256), 0, s, y, n, c0, c1, c2, wtot);
    return hipGetLastError();
}

hipError_t gfnet_launch_adam(float *w, float *m, float *v, uint16_t *wb, const float *g, float lr, float bc1, float bc2,
                             hipStream_t s)
{
    hipLaunchKernelGGL(adam_kernel, dim3((N_PARAMS + 255) / 256), dim3(256), 0, s, w, m, v, wb, g, lr, bc1, bc2);
    return hipGetLastError();
}

hipError_t gfnet_launch_to_bf16(const float *w, uint16_t *wb, int n, hipStream_t s)
{
    hipLaunchKernelGGL(to_bf16_kernel, dim3((n + 255) / 256), dim3(256), 0, s, w, wb, n);
    return hipGetLastError();
}

template <typename RS>
static hipError_t launch_image(const RS *q, const RS *b, int64_t cap, int m, const int32_t *map, const FeatLevel *lv,
                               const FeatLevel &fin, int Lf, float *img, hipStream_t s)
{
    dim3 grid((fin.nx + 255) / 256, fin.ny);
    hipLaunchKernelGGL(image_kernel<RS>, grid, dim3(256), 0, s, q, b, cap, m, map, lv, Lf, fin.nx, fin.ny,
                       img + fin.img_off);
    return hipGetLastError();
}

hipError_t gfnet_launch_image_f32(const float *q, const float *b, int64_t cap, int m, const int32_t *map,
                                  const FeatLevel *lv, const FeatLevel &fin, int Lf, float *img, hipStream_t s)
{
    return launch_image<float>(q, b, cap, m, map, lv, fin, Lf, img, s);
}

hipError_t gfnet_launch_image_f64(const double *q, const double *b, int64_t cap, int m, const int32_t *map,
                                  const FeatLevel *lv, const FeatLevel &fin, int Lf, float *img, hipStream_t s)
{
    return launch_image<double>(q, b, cap, m, map, lv, fin, Lf, img, s);
}

hipError_t gfnet_launch_pyramid(const float *fine, int fnx, int fny, float *coarse, int cnx, int cny, hipStream_t s)
{
    dim3 grid((cnx + 255) / 256, cny);
    hipLaunchKernelGGL(pyramid_kernel, grid, dim3(256), 0, s, fine, fnx, fny, coarse, cnx, cny);
    return hipGetLastError();
}

hipError_t gfnet_launch_tiles(const float *img, const FeatLevel *lv, const int32_t *leaf_lij, int n, float *featf,
                              uint16_t *featb, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(tile_kernel, dim3(n), dim3(256), 0, s, img, lv, leaf_lij, featf, featb);
    return hipGetLastError();
}
