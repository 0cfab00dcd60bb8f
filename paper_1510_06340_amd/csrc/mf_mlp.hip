// mf_mlp.hip -- the learned con2prim seed: a 2 -> 64 -> 64 -> 1 tanh MLP on
// gfx950 with bfloat16 weights and FP32 accumulation.
//
// The 64 x 64 hidden layer runs on the matrix cores
// (gfx950's v_mfma_f32_16x16x32_bf16: A 16x32 (M x K), B 32x16 (K x N), each
// lane holding 8 K values; lane l holds A[l % 16][8 (l / 16) + i] and
// B[8 (l / 16) + i][l % 16], i = 0..7; the accumulator holds
// D[4 (l / 16) + i][l % 16], i = 0..3).  Only the K values a lane holds must
// agree between A and B, so a product over samples may take its K slots in
// any order (the weight gradient uses that to feed the accumulator layout of
// the forward pass straight back in as its A operand).
// Seeded con2prim: one wavefront owns 64 states (4 M-tiles), one per lane for
// the Newton solve.  Forward pass and training: one wavefront owns 16 samples
// (1 M-tile), four to a block, so that a block needs a quarter of the LDS and
// a training batch spreads over four times as many compute units; the weight gradient,
// a product over the 16 samples, takes gfx950's K = 16 form
// (v_mfma_f32_16x16x16_bf16: lane l holds A[l % 16][4 (l / 16) + i] and
// B[4 (l / 16) + i][l % 16], i = 0..3).  Layers 1 and 3 (K = 2, N = 1) run
// on the vector ALUs.
//
// Rounding points (the CPU reference applies the same ones):
//   z1 = bf(W1) x + b1, h1 = tanh z1, h1b = bf(h1)
//   z2 = bf(W2) h1b + b2, h2 = tanh z2, y = bf(w3) . h2 + b3
// Training (mean squared error) back-propagates through the same points,
// with dz2 rounded to bf16 as the operand of both dW2 = dz2b^T h1b and
// dh1 = dz2b bf(W2) on the matrix cores.
//
// Parameter block (FP32, contiguous): W1[64][2], b1[64], W2[64][64], b2[64],
// w3[64], b3.
#include <cmath>
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "mf_device.hpp"
#include "mf_mlp.hpp"

namespace mf {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int H = kMlpHidden;
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + 2 * H;
constexpr int OFF_W2 = OFF_B1 + H;
constexpr int OFF_B2 = OFF_W2 + H * H;
constexpr int OFF_W3 = OFF_B2 + H;
constexpr int OFF_B3 = OFF_W3 + H;
static_assert(OFF_B3 + 1 == kMlpParams, "parameter layout");

constexpr int LDA = H + 8;  // padded LDS row (bf16 elements; 16-byte aligned rows for the 8-value reads)

__device__ __forceinline__ unsigned short f2bf(float f)
{
    unsigned int u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even
    return (unsigned short)(u >> 16);
}

__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float(((unsigned int)h) << 16); }

__device__ __forceinline__ float bfr(float f) { return bf2f(f2bf(f)); }

// Eight bf16 values from LDS (16-byte aligned) as a matrix-core operand.
__device__ __forceinline__ bf16x8 lds8(const unsigned short* p) { return __builtin_bit_cast(bf16x8, *(const s16x8*)p); }

__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Shared-memory image of the weights used by the matrix-core layer (16-byte
// aligned rows: the matrix operands are read 8 values at a time).
struct __align__(16) MlpShared {
    unsigned short w2[H * LDA];   // bf(W2)[n][k]
    unsigned short w2t[H * LDA];  // bf(W2)[k][n] (transposed)
    float w1[2 * H];              // bf(W1)
    float b1[H];
    float b2[H];
    float w3[H];                  // bf(w3)
    float b3;
};

__device__ void load_shared(const float* __restrict__ P, MlpShared& s)
{
    for (int i = threadIdx.x; i < H * H; i += blockDim.x) {
        const int n = i / H, k = i % H;
        const unsigned short v = f2bf(P[OFF_W2 + i]);
        s.w2[n * LDA + k] = v;
        s.w2t[k * LDA + n] = v;
    }
    for (int i = threadIdx.x; i < 2 * H; i += blockDim.x) s.w1[i] = bfr(P[OFF_W1 + i]);
    for (int i = threadIdx.x; i < H; i += blockDim.x) {
        s.b1[i] = P[OFF_B1 + i];
        s.b2[i] = P[OFF_B2 + i];
        s.w3[i] = bfr(P[OFF_W3 + i]);
    }
    if (threadIdx.x == 0) s.b3 = P[OFF_B3];
}

// Forward pass of one wavefront over 16 MT samples.  MT = 4: lane l owns
// sample l and computes its 64 hidden units; MT = 1: lane l computes hidden
// units 16 (l / 16) .. 16 (l / 16) + 15 of sample l % 16 (x0, x1: that
// sample's inputs).  sA: this wavefront's [16 MT][LDA] bf16 buffer.  Returns,
// in the matrix-core accumulator layout, z2 (without bias) for the MT x 4
// (M, N) tiles, and y for the samples 16 mt + 4 (l / 16) + i in yv[mt][i]
// (valid in every lane).
template <int MT>
__device__ __forceinline__ void mlp_forward_wave(const MlpShared& s, unsigned short* sA, float x0, float x1,
                                                 f32x4 acc[MT][4], float yv[MT][4])
{
    const int l = threadIdx.x & 63;
    const int r = l & 15, q = l >> 4;
    // layer 1 (VALU): h1b of the lane's sample into its row of sA
    const int row = MT == 4 ? l : r;
    const int h0 = MT == 4 ? 0 : 16 * q, h1 = MT == 4 ? H : 16 * q + 16;
    for (int h = h0; h < h1; h += 2) {
        const float z0 = __builtin_fmaf(s.w1[2 * h], x0, __builtin_fmaf(s.w1[2 * h + 1], x1, 0.0f)) + s.b1[h];
        const float z1 = __builtin_fmaf(s.w1[2 * h + 2], x0, __builtin_fmaf(s.w1[2 * h + 3], x1, 0.0f)) + s.b1[h + 1];
        const unsigned int pk = (unsigned int)f2bf(tanhf(z0)) | ((unsigned int)f2bf(tanhf(z1)) << 16);
        *(unsigned int*)&sA[row * LDA + h] = pk;
    }
    __syncthreads();
    // layer 2 (matrix cores): z2[s][n] = sum_k h1b[s][k] bf(W2)[n][k]
    for (int mt = 0; mt < MT; mt++) {
        for (int nt = 0; nt < 4; nt++) acc[mt][nt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        for (int kt = 0; kt < 2; kt++) {
            const bf16x8 a = lds8(&sA[(mt * 16 + r) * LDA + kt * 32 + 8 * q]);
            for (int nt = 0; nt < 4; nt++)
                acc[mt][nt] = mfma32(a, lds8(&s.w2[(nt * 16 + r) * LDA + kt * 32 + 8 * q]), acc[mt][nt]);
        }
    }
    // layer 3 (VALU): y[s] = sum_n bf(w3)[n] tanh(z2[s][n] + b2[n]) + b3
    for (int mt = 0; mt < MT; mt++) {
        float part[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int nt = 0; nt < 4; nt++) {
            const int n = nt * 16 + r;
            for (int i = 0; i < 4; i++) part[i] = __builtin_fmaf(s.w3[n], tanhf(acc[mt][nt][i] + s.b2[n]), part[i]);
        }
        for (int i = 0; i < 4; i++) {
            float v = part[i];
            for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, 64);  // sum over the 16 lanes of the row group
            yv[mt][i] = v + s.b3;
        }
    }
}

// y = MLP(X) for B samples (X row-major B x 2).
// (16 MT samples per wavefront, four wavefronts to a block.)
template <int MT>
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ P, const float* __restrict__ X,
                                                     int64_t B, float* __restrict__ y)
{
    __shared__ MlpShared s;
    __shared__ __align__(16) unsigned short sA[4][16 * MT * LDA];
    load_shared(P, s);
    __syncthreads();
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int r = l & 15, q = l >> 4;
    const int64_t base = ((int64_t)blockIdx.x * 4 + w) * (16 * MT);
    const int64_t smp = base + (MT == 4 ? l : r);
    const float x0 = smp < B ? X[2 * smp] : 0.0f;
    const float x1 = smp < B ? X[2 * smp + 1] : 0.0f;
    f32x4 acc[MT][4];
    float yv[MT][4];
    mlp_forward_wave<MT>(s, sA[w], x0, x1, acc, yv);
    if (r == 0) {
        for (int mt = 0; mt < MT; mt++)
            for (int i = 0; i < 4; i++) {
                const int64_t o = base + mt * 16 + 4 * q + i;
                if (o < B) y[o] = yv[mt][i];
            }
    }
}

// Forward + backward of the mean squared error for B samples.  A block of
// four wavefronts owns 64 samples, 16 per wavefront; each wavefront's partial
// gradient (kMlpParams floats and its squared-error sum) goes to LDS, and the
// block writes their sum (in a fixed order) into part[block][kMlpParams + 1].
__global__ __launch_bounds__(256) void k_mlp_grad(const float* __restrict__ P, const float* __restrict__ X,
                                                  const float* __restrict__ T, int64_t B, float* __restrict__ part)
{
    __shared__ MlpShared s;
    __shared__ __align__(16) unsigned short sA[4][16 * LDA];   // h1b per wavefront ([s][k])
    __shared__ __align__(16) unsigned short sD[4][16 * LDA];   // dz2b per wavefront ([s][n])
    __shared__ float sX[4][16][2];
    __shared__ float red[4][kMlpParams + 1];                   // the wavefronts' partial gradients
    load_shared(P, s);
    __syncthreads();
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int r = l & 15, q = l >> 4;
    const int64_t base = ((int64_t)blockIdx.x * 4 + w) * 16;
    const int64_t smp = base + r;   // lanes r, r + 16, r + 32, r + 48 share sample r
    const bool valid = smp < B;
    const float x0 = valid ? X[2 * smp] : 0.0f;
    const float x1 = valid ? X[2 * smp + 1] : 0.0f;
    if (q == 0) {
        sX[w][r][0] = x0;
        sX[w][r][1] = x1;
    }
    f32x4 acc[1][4];
    float yv[1][4];
    mlp_forward_wave<1>(s, sA[w], x0, x1, acc, yv);

    // dy for the samples 4 q + i of this lane's accumulator rows; padding samples get 0
    float dy[4];
    float sq = 0.0f;
    for (int i = 0; i < 4; i++) {
        const int64_t o = base + 4 * q + i;
        const float d = o < B ? yv[0][i] - T[o] : 0.0f;
        dy[i] = 2.0f * d / (float)B;
        if (r == 0) sq += d * d;
    }
    // dz2 = dy w3b (1 - h2^2) in the accumulator layout; dw3, db2 partials per column n
    float gw3[4] = {0, 0, 0, 0}, gb2[4] = {0, 0, 0, 0};
    bf16x4 dzA[4];  // dz2b as the A operand of dW2 (rows n, K = samples): the same lane layout
    for (int nt = 0; nt < 4; nt++) {
        const int n = nt * 16 + r;
        short v[4];
        for (int i = 0; i < 4; i++) {
            const float h2 = tanhf(acc[0][nt][i] + s.b2[n]);
            const float dz = dy[i] * s.w3[n] * (1.0f - h2 * h2);
            gw3[nt] = __builtin_fmaf(dy[i], h2, gw3[nt]);
            gb2[nt] += dz;
            const unsigned short b = f2bf(dz);
            v[i] = (short)b;
            sD[w][(4 * q + i) * LDA + n] = b;
        }
        dzA[nt] = bf16x4{v[0], v[1], v[2], v[3]};
    }
    __syncthreads();

    float* out = red[w];
    // dW2[n][k] = sum_s dz2b[s][n] h1b[s][k]: A = dz2b^T (the lane's K slots are its
    // accumulator rows, samples 4 q + i), B[s][k] = h1b from sA; one K = 16 instruction
    for (int nt = 0; nt < 4; nt++)
        for (int kt = 0; kt < 4; kt++) {
            short v[4];
            for (int i = 0; i < 4; i++) v[i] = (short)sA[w][(4 * q + i) * LDA + kt * 16 + r];
            const f32x4 g = mfma16(dzA[nt], bf16x4{v[0], v[1], v[2], v[3]}, f32x4{0.0f, 0.0f, 0.0f, 0.0f});
            for (int i = 0; i < 4; i++) out[OFF_W2 + (nt * 16 + 4 * q + i) * H + kt * 16 + r] = g[i];
        }
    // dh1[s][k] = sum_n dz2b[s][n] bf(W2)[n][k]: A from sD (rows s), B[n][k] = w2t[k][n]
    float gw1[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}}, gb1[4] = {0, 0, 0, 0};
    for (int kt = 0; kt < 4; kt++) {
        f32x4 g = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int nk = 0; nk < 2; nk++)
            g = mfma32(lds8(&sD[w][r * LDA + nk * 32 + 8 * q]), lds8(&s.w2t[(kt * 16 + r) * LDA + nk * 32 + 8 * q]),
                       g);
        // dz1 = dh1 (1 - h1^2), with h1 recomputed from the sample's x (padding samples have dz2 = 0)
        const int k = kt * 16 + r;
        for (int i = 0; i < 4; i++) {
            const int sl = 4 * q + i;
            const float xa = sX[w][sl][0], xb = sX[w][sl][1];
            const float z1 = __builtin_fmaf(s.w1[2 * k], xa, __builtin_fmaf(s.w1[2 * k + 1], xb, 0.0f)) + s.b1[k];
            const float h1 = tanhf(z1);
            const float dz1 = g[i] * (1.0f - h1 * h1);
            gw1[kt][0] = __builtin_fmaf(dz1, xa, gw1[kt][0]);
            gw1[kt][1] = __builtin_fmaf(dz1, xb, gw1[kt][1]);
            gb1[kt] += dz1;
        }
    }
    // column sums over the 4 row groups (lanes r, r + 16, r + 32, r + 48)
    for (int nt = 0; nt < 4; nt++) {
        for (int o = 16; o < 64; o <<= 1) {
            gw3[nt] += __shfl_xor(gw3[nt], o, 64);
            gb2[nt] += __shfl_xor(gb2[nt], o, 64);
            gw1[nt][0] += __shfl_xor(gw1[nt][0], o, 64);
            gw1[nt][1] += __shfl_xor(gw1[nt][1], o, 64);
            gb1[nt] += __shfl_xor(gb1[nt], o, 64);
        }
    }
    for (int o = 1; o < 64; o <<= 1) sq += __shfl_xor(sq, o, 64);
    if (q == 0) {
        for (int nt = 0; nt < 4; nt++) {
            const int n = nt * 16 + r;
            out[OFF_W3 + n] = gw3[nt];
            out[OFF_B2 + n] = gb2[nt];
            out[OFF_W1 + 2 * n] = gw1[nt][0];
            out[OFF_W1 + 2 * n + 1] = gw1[nt][1];
            out[OFF_B1 + n] = gb1[nt];
        }
    }
    // db3 = sum dy (one value per sample: lanes with r == 0 hold 4 samples each)
    float db3 = 0.0f;
    if (r == 0)
        for (int i = 0; i < 4; i++) db3 += dy[i];
    for (int o = 1; o < 64; o <<= 1) db3 += __shfl_xor(db3, o, 64);
    if (l == 0) {
        out[OFF_B3] = db3;
        out[kMlpParams] = sq;
    }
    __syncthreads();
    // the block's partial: the four wavefronts' sums in a fixed order
    float* dst = part + (int64_t)blockIdx.x * (kMlpParams + 1);
    for (int i = threadIdx.x; i <= kMlpParams; i += blockDim.x) dst[i] = ((red[0][i] + red[1][i]) + red[2][i]) + red[3][i];
}

// grad[p] = sum over blocks of part[w][p] (fixed order); loss = sum sq / B.
// The partials are loaded kBatch at a time before they are added (in order),
// so their latencies overlap: a training batch has few wavefronts of partials
// per thread, and one load in flight at a time left the kernel latency-bound.
__global__ void k_mlp_reduce(const float* __restrict__ part, int nwaves, int64_t B, float* __restrict__ grad,
                             float* __restrict__ loss)
{
    constexpr int kBatch = 16;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kMlpParams) return;
    const float* col = part + p;
    float acc = 0.0f;
    int w = 0;
    for (; w + kBatch <= nwaves; w += kBatch) {
        float x[kBatch];
#pragma unroll
        for (int i = 0; i < kBatch; i++) x[i] = col[(int64_t)(w + i) * (kMlpParams + 1)];
#pragma unroll
        for (int i = 0; i < kBatch; i++) acc += x[i];
    }
    for (; w < nwaves; w++) acc += col[(int64_t)w * (kMlpParams + 1)];
    if (p < kMlpParams) grad[p] = acc;
    else if (loss) *loss = acc / (float)B;
}

// Adam (Kingma & Ba 2015) on the FP32 master parameters.
__global__ void k_mlp_adam(float* __restrict__ P, const float* __restrict__ g, float* __restrict__ m,
                           float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------
// Seeded con2prim over n states with the tabulated EoS.  mode 1: the initial
// guess comes from the MLP on (ln E, |M|/E), evaluated on the matrix cores
// for the wavefront's 64 states (ln e, or the bracket fraction); mode 2: the
// conformal (p = e/3) closed form.  The guess starts the same safeguarded
// Newton solve as the plain one if it lies inside the bracket, else the solve
// starts at the midpoint (counted as a fallback).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_con2prim_seeded(C2PArgs<double> a, EosTable eos, const float* __restrict__ P,
                                                         SeedNorm nrm, int mode)
{
    __shared__ MlpShared s;
    __shared__ __align__(16) unsigned short sA[4][64 * LDA];
    __shared__ float sy[4][64];
    __shared__ double eos_cache[EosTable::kCacheDoubles];
    eos.bind_cache(eos_cache);
    if (mode == 1) load_shared(P, s);
    __syncthreads();
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < a.n;
    double E = 1.0, Mx = 0.0, My = 0.0, Mz = 0.0;
    if (valid) {
        E = a.U[0][i]; Mx = a.U[1][i]; My = a.U[2][i]; Mz = a.U[3][i];
    }
    double M2 = Mx * Mx + My * My + Mz * Mz;
    Counts cnt;
    const bool ok = eos.fixup(E, Mx, My, Mz, M2, cnt);
    if (!ok) {
        E = 1.0; Mx = 0.0; My = 0.0; Mz = 0.0; M2 = 0.0;
    }
    float y = 0.0f;
    if (mode == 1) {
        const float x0 = (__builtin_amdgcn_logf((float)E) * 0.69314718f - nrm.in_shift[0]) * nrm.in_scale[0];
        const float x1 = ((float)(sqrt(M2) / E) - nrm.in_shift[1]) * nrm.in_scale[1];
        f32x4 acc[4][4];
        float yv[4][4];
        mlp_forward_wave<4>(s, sA[w], x0, x1, acc, yv);
        if ((l & 15) == 0)
            for (int mt = 0; mt < 4; mt++)
                for (int k = 0; k < 4; k++) sy[w][mt * 16 + 4 * (l >> 4) + k] = yv[mt][k];
        __syncthreads();
        y = sy[w][l];
    }
    const double q = M2 * Math<double>::rcp(E);
    const double lo = E - q;
    double e_start = E;
    if (M2 != 0.0) {
        double e0;
        if (mode == 1) {
            const double pred = (double)(y * nrm.out_scale + nrm.out_shift);
            e0 = nrm.output == 1 ? E - pred * q : exp(pred);
        } else {
            const double c = 1.0 / 3.0, b = 1.0 + c;
            e0 = E - 2.0 * M2 / (b * E + sqrt(b * b * E * E - 4.0 * c * M2));
        }
        e_start = EosTable::seeded_start(E, lo, e0, cnt);
    }
    double p, dp;
    const double e = eos.solve(E, M2, lo, e_start, p, dp, cnt);
    const double iw = Math<double>::rcp(E + p);
    if (valid) {
        if (ok) {
            a.prim[0][i] = e; a.prim[1][i] = p;
            a.prim[2][i] = Mx * iw; a.prim[3][i] = My * iw; a.prim[4][i] = Mz * iw;
        } else {
            a.prim[0][i] = 0.0; a.prim[1][i] = 0.0; a.prim[2][i] = 0.0; a.prim[3][i] = 0.0; a.prim[4][i] = 0.0;
        }
        if (a.iters) a.iters[i] = (int32_t)cnt.iters;
    }
    if (!valid) cnt = Counts();
    // counters: one atomic per wavefront and counter
    unsigned int c[4] = {cnt.floor_, cnt.bad, cnt.iters, cnt.fallback};
    for (int k = 0; k < 4; k++)
        for (int o = 32; o > 0; o >>= 1) c[k] += __shfl_xor(c[k], o, 64);
    if (l == 0) {
        if (c[0]) atomicAdd(&a.stats[ST_FLOOR], (unsigned long long)c[0]);
        if (c[1]) atomicAdd(&a.stats[ST_BAD], (unsigned long long)c[1]);
        if (c[2]) atomicAdd(&a.stats[ST_ITERS], (unsigned long long)c[2]);
        if (c[3]) atomicAdd(&a.stats[ST_FALLBACK], (unsigned long long)c[3]);
    }
}

hipError_t con2prim_seeded(int64_t n, hipStream_t s, const C2PArgs<double>& a, const EosTable& eos, const float* P,
                           const SeedNorm& nrm, int mode)
{
    const int64_t nb = (n + 255) / 256;
    hipLaunchKernelGGL(k_con2prim_seeded, dim3((unsigned)nb), dim3(256), 0, s, a, eos, P, nrm, mode);
    return hipGetLastError();
}

hipError_t mlp_forward(const float* P, const float* X, int64_t B, float* y, hipStream_t s)
{
    if (B <= 0) return hipSuccess;
    // 16 samples per wavefront: 29 KB of LDS per block (five blocks per compute unit,
    // against two with 64 samples per wavefront), 8.8 against 7.2 G samples/s
    const int64_t blocks = (B + 63) / 64;
    hipLaunchKernelGGL((k_mlp_forward<1>), dim3((unsigned)blocks), dim3(256), 0, s, P, X, B, y);
    return hipGetLastError();
}

int64_t mlp_grad_partials(int64_t B) { return (B + 63) / 64; }   // one per block of 64 samples

hipError_t mlp_grad(const float* P, const float* X, const float* T, int64_t B, float* part, float* grad, float* loss,
                    hipStream_t s)
{
    if (B <= 0) return hipErrorInvalidValue;
    const int64_t blocks = mlp_grad_partials(B);
    hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)blocks), dim3(256), 0, s, P, X, T, B, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kMlpParams + 1 + 255) / 256), dim3(256), 0, s, part, (int)blocks, B,
                       grad, loss);
    return hipGetLastError();
}

hipError_t mlp_adam(float* P, const float* g, float* m, float* v, int step, float lr, float b1, float b2, float eps,
                    hipStream_t s)
{
    // bias corrections 1 - beta^step in double (1 - beta^step cancels badly in float for beta near 1)
    const float c1 = (float)(-std::expm1((double)step * std::log1p(-(1.0 - (double)b1))));
    const float c2 = (float)(-std::expm1((double)step * std::log1p(-(1.0 - (double)b2))));
    hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, P, g, m, v, kMlpParams, lr, b1,
                       b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace mf
