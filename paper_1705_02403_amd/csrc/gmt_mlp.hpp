// gmt_mlp.hpp -- device kernels of the learned sampler (a conditional VAE
// whose encoder and decoder are 3-layer MLPs of width 256): a BF16 GEMM on
// the gfx950 matrix cores with fused bias / ReLU epilogue, the ReLU and bias
// backward, the CVAE loss and reparameterisation, Adam, and the step that
// turns raw decoder outputs into grid-quantised states outside the obstacles.
//
// BF16 values are carried as their 16-bit patterns (unsigned short); FP32
// to BF16 rounds to nearest even.  Every GEMM accumulates in FP32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gmt_mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float f) {
    unsigned int u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);                                                  // nearest even
    return (unsigned short)(u >> 16);
}

__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

// ---------------------------------------------------------------------------
// GEMM: C[M][N] = op(A)[M][K] op(B)[K][N] (+ bias[N]) (ReLU), FP32 accumulate.
//  TA = false: A(m,k) = A[m*lda + k]      TA = true: A(m,k) = A[k*lda + m]
//  TB = false: B(k,n) = B[k*ldb + n]      TB = true: B(k,n) = B[n*ldb + k]
// Writes FP32 (C) and/or BF16 (Cb) with leading dimension ldc.
// grid (ceil(M/64), ceil(N/64)): row tiles along x, which has no small limit.
// Requirements (checked on the host): K, lda, ldb multiples of 8; M (when TA)
// and N (when !TB) multiples of 8; A and B 16-byte aligned.
//
// A 256-thread workgroup computes a 64x64 tile of C; each of its four waves a
// 32x32 quarter as 2x2 blocks of the 16x16x32 BF16 MFMA.  Per step of 32 in K
// both operand tiles are staged in LDS as [row][k] with rows padded to 40
// elements (80 bytes) so that the 16-byte fragment reads of a wave spread
// over the banks.
// ---------------------------------------------------------------------------
#define MLP_T 64
#define MLP_KT 32
#define MLP_KP 40

// stage a 64 x 32 tile (rows r0.., k0..) into dst[r * MLP_KP + k]; rows or
// k beyond (R, K) read as zero.  CK: element (r, k) at src[r*ld + k] (k
// contiguous); otherwise at src[k*ld + r] (r contiguous).
template <bool CK>
__device__ __forceinline__ void stage_tile(const unsigned short *__restrict__ src, int ld, int R, int K, int r0,
                                           int k0, int tid, unsigned short *dst) {
    if (CK) {
        const int r = tid >> 2, k8 = (tid & 3) * 8;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (r0 + r < R && k0 + k8 < K) v = *(const uint4 *)(src + (size_t)(r0 + r) * ld + k0 + k8);
        *(uint4 *)(dst + r * MLP_KP + k8) = v;
    } else {
        const int k = tid >> 3, r8 = (tid & 7) * 8;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (k0 + k < K && r0 + r8 < R) v = *(const uint4 *)(src + (size_t)(k0 + k) * ld + r0 + r8);
        const unsigned short *e = (const unsigned short *)&v;
#pragma unroll
        for (int j = 0; j < 8; ++j) dst[(r8 + j) * MLP_KP + k] = e[j];
    }
}

template <bool TA, bool TB>
__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, const unsigned short *__restrict__ A, int lda,
                                              const unsigned short *__restrict__ B, int ldb,
                                              const float *__restrict__ bias, int relu, float *__restrict__ C,
                                              unsigned short *__restrict__ Cb, int ldc) {
    __shared__ __align__(16) unsigned short As[MLP_T * MLP_KP];
    __shared__ __align__(16) unsigned short Bs[MLP_T * MLP_KP];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.x * MLP_T, n0 = blockIdx.y * MLP_T;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += MLP_KT) {
        __syncthreads();  // previous step's fragment reads are done
        stage_tile<!TA>(A, lda, M, K, m0, k0, tid, As);
        stage_tile<TB>(B, ldb, N, K, n0, k0, tid, Bs);
        __syncthreads();
        bf16x8 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            a[i] = *(const bf16x8 *)(As + (wm + 16 * i + fr) * MLP_KP + fk);
            b[i] = *(const bf16x8 *)(Bs + (wn + 16 * i + fr) * MLP_KP + fk);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    // 16x16 result block: lane holds rows 4*(lane/16) + q, column lane % 16
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + wn + 16 * j + fr;
            if (n >= N) continue;
            const float bn = bias ? bias[n] : 0.f;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = m0 + wm + 16 * i + (lane >> 4) * 4 + q;
                if (m >= M) continue;
                float v = acc[i][j][q] + bn;
                if (relu) v = fmaxf(v, 0.f);
                if (C) C[(size_t)m * ldc + n] = v;
                if (Cb) Cb[(size_t)m * ldc + n] = f2bf(v);
            }
        }
}

// ---------------------------------------------------------------------------
// activation backward: dZ = dY * [Y > 0] (relu) or dY, stored as BF16; the
// bias gradient sum_m dZ[m][n] in two fixed-order passes (per 256-row chunk,
// then over chunks), so it is deterministic.
// grid (ceil(M/256), ceil(N/64)), 256 threads; part is [chunks][N].
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_act_bwd(int M, int N, const float *__restrict__ dY, int ldy,
                                                 const unsigned short *__restrict__ Y, int ldyy, int relu,
                                                 unsigned short *__restrict__ dZ, int ldz, float *__restrict__ part) {
    __shared__ float red[4][64];
    const int c = threadIdx.x & 63, rg = threadIdx.x >> 6;
    const int n = blockIdx.y * 64 + c;
    float s = 0.f;
    if (n < N) {
        const int mb = blockIdx.x * 256;
        for (int it = 0; it < 64; ++it) {
            const int m = mb + rg + 4 * it;
            if (m >= M) break;
            float g = dY[(size_t)m * ldy + n];
            if (relu && !(bf2f(Y[(size_t)m * ldyy + n]) > 0.f)) g = 0.f;
            dZ[(size_t)m * ldz + n] = f2bf(g);
            s += g;
        }
    }
    red[rg][c] = s;
    __syncthreads();
    if (rg == 0 && n < N) part[(size_t)blockIdx.x * N + n] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
}

__global__ void k_colsum(int N, int chunks, const float *__restrict__ part, float *__restrict__ out) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int c = 0; c < chunks; ++c) s += part[(size_t)c * N + n];
    out[n] = s;
}

// ---------------------------------------------------------------------------
// CVAE pieces.  Encoder output E[b][0..5] = mu, E[b][6..11] = log variance;
// decoder output D[b][0..5] = reconstruction; rows of 16 (GMT_MLP_OUT).
// ---------------------------------------------------------------------------
#define MLP_IN 416    // padded input width
#define MLP_COND 396  // condition features
#define MLP_COND0 8   // first condition column of an input row
#define MLP_OUT 16    // padded output width
#define MLP_X 6       // state dimension

// training rows: x (encoder) and the condition of the waypoint's problem;
// the decoder row gets the same condition (its z columns come later)
__global__ void k_gather(int B, const int *__restrict__ rows, const int *__restrict__ owner,
                         const float *__restrict__ cond, const float *__restrict__ targ, unsigned short *__restrict__ Xe,
                         unsigned short *__restrict__ Xd, float *__restrict__ T) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)B * MLP_IN) return;
    const int b = (int)(t / MLP_IN), c = (int)(t % MLP_IN);
    const int row = rows[b];
    unsigned short e = 0, d = 0;
    if (c < MLP_X) {
        const float x = targ[(size_t)row * MLP_X + c];
        e = f2bf(x);
        T[(size_t)b * MLP_X + c] = x;
    } else if (c >= MLP_COND0 && c < MLP_COND0 + MLP_COND) {
        e = d = f2bf(cond[(size_t)owner[row] * MLP_COND + (c - MLP_COND0)]);
    }
    Xe[t] = e;
    Xd[t] = d;
}

// z = mu + exp(logvar / 2) * eps into the decoder rows
__global__ void k_reparam(int B, const float *__restrict__ E, const float *__restrict__ eps,
                          unsigned short *__restrict__ Xd) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B * 8) return;
    const int b = t >> 3, j = t & 7;
    unsigned short v = 0;
    if (j < MLP_X) {
        const float mu = E[(size_t)b * MLP_OUT + j], lv = E[(size_t)b * MLP_OUT + MLP_X + j];
        v = f2bf(mu + expf(0.5f * lv) * eps[(size_t)b * MLP_X + j]);
    }
    Xd[(size_t)b * MLP_IN + j] = v;
}

// per row: reconstruction term 0.5 * w * |D - T|^2 and KL term
// 0.5 * sum(mu^2 + exp(lv) - 1 - lv); gradient of the batch mean w.r.t. D
__global__ void k_cvae_loss(int B, const float *__restrict__ E, const float *__restrict__ D,
                            const float *__restrict__ T, float w, float *__restrict__ dD, float *__restrict__ terms) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const float inv_b = 1.0f / (float)B;
    float rec = 0.f, kl = 0.f;
    for (int j = 0; j < MLP_OUT; ++j) {
        float g = 0.f;
        if (j < MLP_X) {
            const float r = D[(size_t)b * MLP_OUT + j] - T[(size_t)b * MLP_X + j];
            rec += r * r;
            g = w * r * inv_b;
            const float mu = E[(size_t)b * MLP_OUT + j], lv = E[(size_t)b * MLP_OUT + MLP_X + j];
            kl += mu * mu + expf(lv) - 1.f - lv;
        }
        dD[(size_t)b * MLP_OUT + j] = g;
    }
    terms[2 * b] = 0.5f * w * rec;
    terms[2 * b + 1] = 0.5f * kl;
}

// batch means of the two loss terms, one workgroup, fixed order
__global__ void __launch_bounds__(256) k_loss_mean(int B, const float *__restrict__ terms, float *__restrict__ out) {
    __shared__ float r[2][256];
    float a = 0.f, k = 0.f;
    for (int b = threadIdx.x; b < B; b += 256) {
        a += terms[2 * b];
        k += terms[2 * b + 1];
    }
    r[0][threadIdx.x] = a;
    r[1][threadIdx.x] = k;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            r[0][threadIdx.x] += r[0][threadIdx.x + s];
            r[1][threadIdx.x] += r[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = r[0][0] / (float)B;
        out[1] = r[1][0] / (float)B;
    }
}

// gradient at the encoder output: through z (dz = decoder input gradient,
// rows of 8) and the KL term weighted by beta
__global__ void k_head_grad(int B, const float *__restrict__ E, const float *__restrict__ eps,
                            const float *__restrict__ dz, float beta, float *__restrict__ dE) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B * MLP_OUT) return;
    const int b = t / MLP_OUT, j = t % MLP_OUT;
    const float inv_b = 1.0f / (float)B;
    float g = 0.f;
    if (j < MLP_X) {
        g = dz[(size_t)b * 8 + j] + beta * E[(size_t)b * MLP_OUT + j] * inv_b;
    } else if (j < 2 * MLP_X) {
        const int a = j - MLP_X;
        const float lv = E[(size_t)b * MLP_OUT + j];
        g = dz[(size_t)b * 8 + a] * 0.5f * expf(0.5f * lv) * eps[(size_t)b * MLP_X + a] +
            beta * 0.5f * (expf(lv) - 1.f) * inv_b;
    }
    dE[t] = g;
}

// Adam with bias correction factors c1 = 1/(1-b1^t), c2 = 1/(1-b2^t); keeps
// the BF16 copy of the parameters in step
__global__ void k_adam(long long n, float *__restrict__ P, const float *__restrict__ G, float *__restrict__ Mo,
                       float *__restrict__ Vo, unsigned short *__restrict__ Pb, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = G[i];
    const float m = b1 * Mo[i] + (1.f - b1) * g;
    const float v = b2 * Vo[i] + (1.f - b2) * g * g;
    Mo[i] = m;
    Vo[i] = v;
    const float p = P[i] - lr * (m * c1) / (sqrtf(v * c2) + eps);
    P[i] = p;
    Pb[i] = f2bf(p);
}

__global__ void k_to_bf16(long long n, const float *__restrict__ src, unsigned short *__restrict__ dst) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = f2bf(src[i]);
}

__global__ void k_fill_f32(long long n, float *__restrict__ p, float v) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// inference
// ---------------------------------------------------------------------------
// first-layer pre-activation shared by every sample of one query: the
// condition's part of W1 x + b1 (condition rounded to BF16 as in training).
// One wave per output: lanes read the weight row coalesced, then reduce.
__global__ void __launch_bounds__(256) k_cond_bias(int H, const unsigned short *__restrict__ W1,
                                                   const float *__restrict__ b1, const float *__restrict__ cond,
                                                   float *__restrict__ h0) {
    const int n = (blockIdx.x * blockDim.x + threadIdx.x) / 64, lane = threadIdx.x & 63;
    if (n >= H) return;
    float s = 0.f;
    for (int k = lane; k < MLP_COND; k += 64)
        s += bf2f(W1[(size_t)n * MLP_IN + MLP_COND0 + k]) * bf2f(f2bf(cond[k]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) h0[n] = s + b1[n];
}

// prior draws z = eps as BF16 rows of 8
__global__ void k_pack_z(int count, const float *__restrict__ eps, unsigned short *__restrict__ Z) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count * 8) return;
    const int b = t >> 3, j = t & 7;
    Z[t] = j < MLP_X ? f2bf(eps[(size_t)b * MLP_X + j]) : (unsigned short)0;
}

// Raw decoder output u (6 values per sample, row stride ldr) -> state:
// position sigmoid(u), velocity w / sqrt(1 + |w|^2) (the open unit ball),
// rounded to the 2^-20 grid in FP64.  A sample with a non-finite value, a
// velocity off the closed unit ball after rounding, or a position in a closed
// box (grid units, [m][lo3 hi3]) is replaced by the caller's fallback sample.
// Output SoA [6][ld].
__global__ void k_finish(int count, const float *__restrict__ raw, int ldr, int m, const int *__restrict__ boxq,
                         const float *__restrict__ fallback, int ldf, float *__restrict__ out, int ld,
                         int *__restrict__ rejected) {
#pragma clang fp contract(off)  // each product and sum rounded on its own, as written
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= count) return;
    double u[6];
    bool bad = false;
    for (int a = 0; a < 6; ++a) {
        u[a] = (double)raw[(size_t)b * ldr + a];
        if (!isfinite(u[a])) bad = true;
    }
    long long q[6] = {0, 0, 0, 0, 0, 0};
    if (!bad) {
        for (int a = 0; a < 3; ++a) q[a] = llrint(1.0 / (1.0 + exp(-u[a])) * 1048576.0);
        const double s = sqrt(1.0 + (u[3] * u[3] + u[4] * u[4] + u[5] * u[5]));
        for (int a = 0; a < 3; ++a) q[3 + a] = llrint(u[3 + a] / s * 1048576.0);
        if (q[3] * q[3] + q[4] * q[4] + q[5] * q[5] > (1ll << 40)) bad = true;
        for (int k = 0; k < m && !bad; ++k) {
            const int *bx = boxq + 6 * k;
            bool in = true;
            for (int a = 0; a < 3; ++a) in = in && q[a] >= bx[a] && q[a] <= bx[3 + a];
            if (in) bad = true;
        }
    }
    if (bad) {
        atomicAdd(rejected, 1);
        for (int a = 0; a < 6; ++a) out[(size_t)a * ld + b] = fallback[(size_t)a * ldf + b];
    } else {
        for (int a = 0; a < 6; ++a) out[(size_t)a * ld + b] = (float)((double)q[a] * (1.0 / 1048576.0));
    }
}

}  // namespace gmt_mlp
