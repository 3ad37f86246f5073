// gmt_sampler.hip -- host side of include/gmt_sampler.h: the BF16 GEMM entry
// point and the learned sampler (training step, decoding, finishing).
//
// Every step of training and inference runs in the kernels of gmt_mlp.hpp on
// the caller's stream; the host only validates arguments, stages small
// inputs through pinned memory and sequences launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/gmt_sampler.h"
#include "gmt_host.hpp"
#include "gmt_mlp.hpp"

using gmt_host::DevBuf;
using gmt_host::dev_alloc;
using gmt_host::dev_free;
using gmt_host::fail;
using namespace gmt_mlp;

namespace {

constexpr int H = GMT_SAMPLER_HIDDEN, IN = GMT_SAMPLER_IN, OUT = GMT_SAMPLER_OUT;
constexpr long long NETP = GMT_SAMPLER_NET_PARAMS, ALLP = GMT_SAMPLER_PARAMS;
static_assert(IN == MLP_IN && OUT == MLP_OUT && GMT_SAMPLER_COND == MLP_COND, "layout constants");

// offsets of one network's tensors in the flat parameter array
struct NetOff {
    long long W1, b1, W2, b2, W3, b3;
};

NetOff net_off(int net) {
    NetOff o;
    o.W1 = net * NETP;
    o.b1 = o.W1 + (long long)H * IN;
    o.W2 = o.b1 + H;
    o.b2 = o.W2 + (long long)H * H;
    o.W3 = o.b2 + H;
    o.b3 = o.W3 + (long long)OUT * H;
    return o;
}

unsigned blocks(long long n, int per) { return (unsigned)((n + per - 1) / per); }

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

gmt_status gemm(bool ta, bool tb, int M, int N, int K, const uint16_t *A, int lda, const uint16_t *B, int ldb,
                const float *bias, bool relu, float *C, uint16_t *Cb, int ldc, hipStream_t s) {
    if (M < 1 || N < 1 || K < 1) return fail(GMT_EINVAL, "gemm: sizes must be >= 1 (M=%d N=%d K=%d)", M, N, K);
    if (!A || !B || (!C && !Cb)) return fail(GMT_EINVAL, "gemm: null operand or output");
    if (K % 8 || lda % 8 || ldb % 8) return fail(GMT_EINVAL, "gemm: K, lda and ldb must be multiples of 8");
    if ((ta && M % 8) || (!tb && N % 8)) return fail(GMT_EINVAL, "gemm: the contiguous dimension must be a multiple of 8");
    if (ldc < N || lda < (ta ? M : K) || ldb < (tb ? K : N)) return fail(GMT_EINVAL, "gemm: leading dimension too small");
    if (!aligned16(A) || !aligned16(B)) return fail(GMT_EINVAL, "gemm: operands must be 16-byte aligned");
    const dim3 grid(blocks(M, MLP_T), blocks(N, MLP_T)), block(256);
    const unsigned short *a = (const unsigned short *)A, *b = (const unsigned short *)B;
    unsigned short *cb = (unsigned short *)Cb;
    const int r = relu ? 1 : 0;
    if (!ta && tb) k_gemm<false, true><<<grid, block, 0, s>>>(M, N, K, a, lda, b, ldb, bias, r, C, cb, ldc);
    else if (!ta && !tb) k_gemm<false, false><<<grid, block, 0, s>>>(M, N, K, a, lda, b, ldb, bias, r, C, cb, ldc);
    else if (ta && !tb) k_gemm<true, false><<<grid, block, 0, s>>>(M, N, K, a, lda, b, ldb, bias, r, C, cb, ldc);
    else k_gemm<true, true><<<grid, block, 0, s>>>(M, N, K, a, lda, b, ldb, bias, r, C, cb, ldc);
    HIPCHK(hipGetLastError());
    return GMT_OK;
}

// pinned staging for small host inputs; the event guards reuse of the buffer
struct Stage {
    void *h = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;

    gmt_status upload(const void *src, size_t bytes, void *dst, hipStream_t s) {
        if (ev) HIPCHK(hipEventSynchronize(ev));
        if (bytes > cap) {
            if (h) (void)hipHostFree(h);
            h = nullptr;
            cap = 0;
            HIPCHK(hipHostMalloc(&h, bytes));
            cap = bytes;
        }
        std::memcpy(h, src, bytes);
        HIPCHK(hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, s));
        if (!ev) HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        HIPCHK(hipEventRecord(ev, s));
        return GMT_OK;
    }

    void release() {
        if (ev) {
            (void)hipEventSynchronize(ev);
            (void)hipEventDestroy(ev);
        }
        if (h) (void)hipHostFree(h);
        h = nullptr;
        ev = nullptr;
        cap = 0;
    }
};

// boxes on the 2^-20 grid as integers; false if a coordinate is off the grid
gmt_status boxes_to_grid(const float *boxes, int m, std::vector<int> &q) {
    if (m < 0 || m > GMT_MAX_BOXES) return fail(GMT_EINVAL, "box count %d outside [0, %d]", m, GMT_MAX_BOXES);
    if (m > 0 && !boxes) return fail(GMT_EINVAL, "null boxes");
    q.assign((size_t)std::max(m, 1) * 6, 0);
    for (int k = 0; k < 6 * m; ++k) {
        const double v = (double)boxes[k] * 1048576.0;
        if (!(v == std::floor(v)) || v < -1048576.0 || v > 2097152.0)
            return fail(GMT_EINVAL, "box %d: coordinate off the 2^-20 grid or out of range", k / 6);
        q[k] = (int)v;
    }
    return GMT_OK;
}

gmt_status finish_launch(const float *raw, int ldr, int count, const int *boxq, int m, const float *fallback, int ldf,
                         float *out, int ld, int *rej, hipStream_t s) {
    k_finish<<<blocks(count, 256), 256, 0, s>>>(count, raw, ldr, m, boxq, fallback, ldf, out, ld, rej);
    HIPCHK(hipGetLastError());
    return GMT_OK;
}

gmt_status check_finish_args(const float *raw, int ldr, int count, const float *fallback, int ldf, const float *out,
                             int ld) {
    if (count < 1 || count > (1 << 24)) return fail(GMT_EINVAL, "count %d outside [1, 2^24]", count);
    if (!raw || !fallback || !out) return fail(GMT_EINVAL, "null raw, fallback or output");
    if (ldr < 6 || ldf < count || ld < count) return fail(GMT_EINVAL, "leading dimension too small");
    return GMT_OK;
}

}  // namespace

extern "C" gmt_status gmt_gemm_bf16(int32_t trans_a, int32_t trans_b, int32_t M, int32_t N, int32_t K,
                                    const uint16_t *d_A, int32_t lda, const uint16_t *d_B, int32_t ldb,
                                    const float *d_bias, int32_t relu, float *d_C, uint16_t *d_Cb, int32_t ldc,
                                    void *stream) {
    return gemm(trans_a != 0, trans_b != 0, M, N, K, d_A, lda, d_B, ldb, d_bias, relu != 0, d_C, d_Cb, ldc,
                (hipStream_t)stream);
}

struct gmt_sampler {
    int device = 0;
    DevBuf P, Pb, G, Mo, Vo;  // FP32 master, BF16 copy, gradients, Adam moments
    long long step = 0;
    // resident training set
    DevBuf cond, targ, owner;
    int nP = 0, nW = 0;
    // training activations for batches of up to `cap` rows
    int cap = 0;
    DevBuf rows, Xe, Xd, H1, H2, G1, G2, E, D, T, dD, dE, dY, dZ, dO, dz, part, terms;
    // inference buffers for up to `icap` samples
    int icap = 0;
    DevBuf icond, h0, Z8, A1, A2, Dout, boxq, rej;
    Stage st_rows, st_cond, st_boxes;
};

namespace {

void free_train(gmt_sampler *s) {
    for (DevBuf *b : {&s->rows, &s->Xe, &s->Xd, &s->H1, &s->H2, &s->G1, &s->G2, &s->E, &s->D, &s->T, &s->dD, &s->dE,
                      &s->dY, &s->dZ, &s->dO, &s->dz, &s->part, &s->terms})
        dev_free(*b, nullptr);
    s->cap = 0;
}

gmt_status ensure_train(gmt_sampler *s, int B, hipStream_t st) {
    if (B <= s->cap) return GMT_OK;
    (void)hipStreamSynchronize(st);
    free_train(s);
    const size_t b = (size_t)B;
    TRY(dev_alloc(s->rows, 4 * b, st));
    TRY(dev_alloc(s->Xe, 2 * b * IN, st));
    TRY(dev_alloc(s->Xd, 2 * b * IN, st));
    TRY(dev_alloc(s->H1, 2 * b * H, st));
    TRY(dev_alloc(s->H2, 2 * b * H, st));
    TRY(dev_alloc(s->G1, 2 * b * H, st));
    TRY(dev_alloc(s->G2, 2 * b * H, st));
    TRY(dev_alloc(s->E, 4 * b * OUT, st));
    TRY(dev_alloc(s->D, 4 * b * OUT, st));
    TRY(dev_alloc(s->T, 4 * b * MLP_X, st));
    TRY(dev_alloc(s->dD, 4 * b * OUT, st));
    TRY(dev_alloc(s->dE, 4 * b * OUT, st));
    TRY(dev_alloc(s->dY, 4 * b * H, st));
    TRY(dev_alloc(s->dZ, 2 * b * H, st));
    TRY(dev_alloc(s->dO, 2 * b * OUT, st));
    TRY(dev_alloc(s->dz, 4 * b * 8, st));
    TRY(dev_alloc(s->part, 4 * (size_t)blocks(B, 256) * H, st));
    TRY(dev_alloc(s->terms, 8 * b, st));
    s->cap = B;
    return GMT_OK;
}

void free_infer(gmt_sampler *s) {
    for (DevBuf *b : {&s->icond, &s->h0, &s->Z8, &s->A1, &s->A2, &s->Dout}) dev_free(*b, nullptr);
    s->icap = 0;
}

gmt_status ensure_infer(gmt_sampler *s, int count, hipStream_t st) {
    if (!s->icond.p) {
        TRY(dev_alloc(s->icond, 4 * MLP_COND, st));
        TRY(dev_alloc(s->h0, 4 * H, st));
        TRY(dev_alloc(s->rej, 4, st));
        TRY(dev_alloc(s->boxq, 4 * (6 * GMT_MAX_BOXES + 8), st));  // boxes, then the zero for the counter
    }
    if (count <= s->icap) return GMT_OK;
    (void)hipStreamSynchronize(st);
    for (DevBuf *b : {&s->Z8, &s->A1, &s->A2, &s->Dout}) dev_free(*b, nullptr);
    const size_t c = (size_t)count;
    TRY(dev_alloc(s->Z8, 2 * c * 8, st));
    TRY(dev_alloc(s->A1, 2 * c * H, st));
    TRY(dev_alloc(s->A2, 2 * c * H, st));
    TRY(dev_alloc(s->Dout, 4 * c * OUT, st));
    s->icap = count;
    return GMT_OK;
}

// dZ (BF16) and the bias gradient from an FP32 upstream gradient
gmt_status act_bwd(gmt_sampler *s, int B, int N, const float *dY, int ldy, const uint16_t *Y, bool relu, uint16_t *dZ,
                   float *db, hipStream_t st) {
    const int chunks = (int)blocks(B, 256);
    k_act_bwd<<<dim3(chunks, blocks(N, 64)), 256, 0, st>>>(B, N, dY, ldy, (const unsigned short *)Y, N, relu ? 1 : 0,
                                                          (unsigned short *)dZ, N, (float *)s->part.p);
    k_colsum<<<blocks(N, 256), 256, 0, st>>>(N, chunks, (const float *)s->part.p, db);
    HIPCHK(hipGetLastError());
    return GMT_OK;
}

// forward of one network over B rows of X: hidden h1, h2 (BF16), output (FP32)
gmt_status net_forward(gmt_sampler *s, int net, int B, const uint16_t *X, uint16_t *h1, uint16_t *h2, float *out,
                       hipStream_t st) {
    const NetOff o = net_off(net);
    const uint16_t *Wb = (const uint16_t *)s->Pb.p;
    const float *P = (const float *)s->P.p;
    TRY(gemm(false, true, B, H, IN, X, IN, Wb + o.W1, IN, P + o.b1, true, nullptr, h1, H, st));
    TRY(gemm(false, true, B, H, H, h1, H, Wb + o.W2, H, P + o.b2, true, nullptr, h2, H, st));
    TRY(gemm(false, true, B, OUT, H, h2, H, Wb + o.W3, H, P + o.b3, false, out, nullptr, OUT, st));
    return GMT_OK;
}

// backward of one network from the FP32 output gradient dOut [B][16]; fills
// its slice of the gradient array; when dz is given, also the gradient of
// the first 8 input columns (the decoder's z)
gmt_status net_backward(gmt_sampler *s, int net, int B, const uint16_t *X, const uint16_t *h1, const uint16_t *h2,
                        const float *dOut, float *dz, hipStream_t st) {
    const NetOff o = net_off(net);
    const uint16_t *Wb = (const uint16_t *)s->Pb.p;
    float *G = (float *)s->G.p;
    uint16_t *dO = (uint16_t *)s->dO.p, *dZ = (uint16_t *)s->dZ.p;
    float *dY = (float *)s->dY.p;
    // output layer
    TRY(act_bwd(s, B, OUT, dOut, OUT, nullptr, false, dO, G + o.b3, st));
    TRY(gemm(true, false, OUT, H, B, dO, OUT, h2, H, nullptr, false, G + o.W3, nullptr, H, st));
    TRY(gemm(false, false, B, H, OUT, dO, OUT, Wb + o.W3, H, nullptr, false, dY, nullptr, H, st));
    // second layer
    TRY(act_bwd(s, B, H, dY, H, h2, true, dZ, G + o.b2, st));
    TRY(gemm(true, false, H, H, B, dZ, H, h1, H, nullptr, false, G + o.W2, nullptr, H, st));
    TRY(gemm(false, false, B, H, H, dZ, H, Wb + o.W2, H, nullptr, false, dY, nullptr, H, st));
    // first layer
    TRY(act_bwd(s, B, H, dY, H, h1, true, dZ, G + o.b1, st));
    TRY(gemm(true, false, H, IN, B, dZ, H, X, IN, nullptr, false, G + o.W1, nullptr, IN, st));
    if (dz) TRY(gemm(false, false, B, 8, H, dZ, H, Wb + o.W1, IN, nullptr, false, dz, nullptr, 8, st));
    return GMT_OK;
}

gmt_status upload_params(gmt_sampler *s, const float *params, hipStream_t st) {
    HIPCHK(hipMemcpyAsync(s->P.p, params, 4 * (size_t)ALLP, hipMemcpyHostToDevice, st));
    k_to_bf16<<<blocks(ALLP, 256), 256, 0, st>>>(ALLP, (const float *)s->P.p, (unsigned short *)s->Pb.p);
    HIPCHK(hipGetLastError());
    return GMT_OK;
}

}  // namespace

extern "C" gmt_status gmt_sampler_create(const float *params, gmt_sampler_t *out) {
    if (!params || !out) return fail(GMT_EINVAL, "null params or output");
    for (long long k = 0; k < ALLP; ++k)
        if (!std::isfinite(params[k])) return fail(GMT_EINVAL, "parameter %lld is not finite", k);
    gmt_sampler *s = new gmt_sampler();
    (void)hipGetDevice(&s->device);
    hipStream_t st = nullptr;
    gmt_status r = GMT_OK;
    for (DevBuf *b : {&s->P, &s->G, &s->Mo, &s->Vo})
        if (r == GMT_OK) r = dev_alloc(*b, 4 * (size_t)ALLP, st);
    if (r == GMT_OK) r = dev_alloc(s->Pb, 2 * (size_t)ALLP, st);
    if (r == GMT_OK) r = upload_params(s, params, st);
    if (r == GMT_OK) {
        for (DevBuf *b : {&s->G, &s->Mo, &s->Vo})
            k_fill_f32<<<blocks(ALLP, 256), 256, 0, st>>>(ALLP, (float *)b->p, 0.f);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
            r = fail(GMT_EDEVICE, "sampler initialisation failed");
    }
    if (r != GMT_OK) {
        gmt_sampler_destroy(s);
        return r;
    }
    *out = s;
    return GMT_OK;
}

extern "C" gmt_status gmt_sampler_get_params(gmt_sampler_t s, float *params) {
    if (!s || !params) return fail(GMT_EINVAL, "null argument");
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(params, s->P.p, 4 * (size_t)ALLP, hipMemcpyDeviceToHost));
    return GMT_OK;
}

extern "C" gmt_status gmt_sampler_get_grads(gmt_sampler_t s, float *grads) {
    if (!s || !grads) return fail(GMT_EINVAL, "null argument");
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(grads, s->G.p, 4 * (size_t)ALLP, hipMemcpyDeviceToHost));
    return GMT_OK;
}

extern "C" gmt_status gmt_sampler_set_data(gmt_sampler_t s, const float *cond, int32_t P, const float *targets,
                                           const int32_t *owner, int32_t W) {
    if (!s || !cond || !targets || !owner) return fail(GMT_EINVAL, "null argument");
    if (P < 1 || W < 1) return fail(GMT_EINVAL, "empty training set");
    for (int k = 0; k < W; ++k)
        if (owner[k] < 0 || owner[k] >= P) return fail(GMT_EINVAL, "owner[%d] = %d outside [0, %d)", k, owner[k], P);
    for (long long k = 0; k < (long long)W * MLP_X; ++k)
        if (!std::isfinite(targets[k])) return fail(GMT_EINVAL, "target value %lld is not finite", k);
    for (long long k = 0; k < (long long)P * MLP_COND; ++k)
        if (!std::isfinite(cond[k])) return fail(GMT_EINVAL, "condition value %lld is not finite", k);
    HIPCHK(hipDeviceSynchronize());
    dev_free(s->cond, nullptr);
    dev_free(s->targ, nullptr);
    dev_free(s->owner, nullptr);
    s->nP = s->nW = 0;
    TRY(dev_alloc(s->cond, 4 * (size_t)P * MLP_COND, nullptr));
    TRY(dev_alloc(s->targ, 4 * (size_t)W * MLP_X, nullptr));
    TRY(dev_alloc(s->owner, 4 * (size_t)W, nullptr));
    HIPCHK(hipMemcpy(s->cond.p, cond, 4 * (size_t)P * MLP_COND, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(s->targ.p, targets, 4 * (size_t)W * MLP_X, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(s->owner.p, owner, 4 * (size_t)W, hipMemcpyHostToDevice));
    s->nP = P;
    s->nW = W;
    return GMT_OK;
}

extern "C" gmt_status gmt_sampler_train_step(gmt_sampler_t s, const int32_t *rows, const float *d_eps, int32_t B,
                                             const gmt_train_opts *opts, float *d_loss, void *stream) {
    if (!s || !rows || !d_eps || !opts) return fail(GMT_EINVAL, "null argument");
    if (s->nW < 1) return fail(GMT_EINVAL, "no training set (gmt_sampler_set_data)");
    if (B < 8 || B > 65536 || B % 8) return fail(GMT_EINVAL, "batch %d must be a multiple of 8 in [8, 65536]", B);
    for (int k = 0; k < B; ++k)
        if (rows[k] < 0 || rows[k] >= s->nW) return fail(GMT_EINVAL, "rows[%d] = %d outside [0, %d)", k, rows[k], s->nW);
    const gmt_train_opts o = *opts;
    if (!(o.lr >= 0.f) || !(o.beta1 >= 0.f && o.beta1 < 1.f) || !(o.beta2 >= 0.f && o.beta2 < 1.f) ||
        !(o.adam_eps > 0.f) || !std::isfinite(o.recon_weight) || !std::isfinite(o.kl_weight))
        return fail(GMT_EINVAL, "bad training options");
    hipStream_t st = (hipStream_t)stream;
    TRY(ensure_train(s, B, st));
    TRY(s->st_rows.upload(rows, 4 * (size_t)B, s->rows.p, st));
    uint16_t *Xe = (uint16_t *)s->Xe.p, *Xd = (uint16_t *)s->Xd.p;
    k_gather<<<blocks((long long)B * IN, 256), 256, 0, st>>>(B, (const int *)s->rows.p, (const int *)s->owner.p,
                                                           (const float *)s->cond.p, (const float *)s->targ.p,
                                                           (unsigned short *)Xe, (unsigned short *)Xd, (float *)s->T.p);
    HIPCHK(hipGetLastError());
    // encoder, reparameterisation, decoder
    TRY(net_forward(s, 0, B, Xe, (uint16_t *)s->H1.p, (uint16_t *)s->H2.p, (float *)s->E.p, st));
    k_reparam<<<blocks(B * 8, 256), 256, 0, st>>>(B, (const float *)s->E.p, d_eps, (unsigned short *)Xd);
    TRY(net_forward(s, 1, B, Xd, (uint16_t *)s->G1.p, (uint16_t *)s->G2.p, (float *)s->D.p, st));
    // loss and its gradient at the decoder output
    k_cvae_loss<<<blocks(B, 256), 256, 0, st>>>(B, (const float *)s->E.p, (const float *)s->D.p,
                                                (const float *)s->T.p, o.recon_weight, (float *)s->dD.p,
                                                (float *)s->terms.p);
    if (d_loss) k_loss_mean<<<1, 256, 0, st>>>(B, (const float *)s->terms.p, d_loss);
    HIPCHK(hipGetLastError());
    // decoder backward (with the gradient at z), head, encoder backward
    TRY(net_backward(s, 1, B, Xd, (const uint16_t *)s->G1.p, (const uint16_t *)s->G2.p, (const float *)s->dD.p,
                     (float *)s->dz.p, st));
    k_head_grad<<<blocks(B * OUT, 256), 256, 0, st>>>(B, (const float *)s->E.p, d_eps, (const float *)s->dz.p,
                                                      o.kl_weight, (float *)s->dE.p);
    HIPCHK(hipGetLastError());
    TRY(net_backward(s, 0, B, Xe, (const uint16_t *)s->H1.p, (const uint16_t *)s->H2.p, (const float *)s->dE.p,
                     nullptr, st));
    // Adam
    s->step += 1;
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)o.beta1, (double)s->step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)o.beta2, (double)s->step)));
    k_adam<<<blocks(ALLP, 256), 256, 0, st>>>(ALLP, (float *)s->P.p, (const float *)s->G.p, (float *)s->Mo.p,
                                             (float *)s->Vo.p, (unsigned short *)s->Pb.p, o.lr, o.beta1, o.beta2,
                                             o.adam_eps, c1, c2);
    HIPCHK(hipGetLastError());
    return GMT_OK;
}

namespace {

gmt_status decode_impl(gmt_sampler *s, const float *cond, const float *d_eps, int count, hipStream_t st) {
    if (!s || !cond || !d_eps) return fail(GMT_EINVAL, "null argument");
    if (count < 1 || count > (1 << 24)) return fail(GMT_EINVAL, "count %d outside [1, 2^24]", count);
    for (int k = 0; k < MLP_COND; ++k)
        if (!std::isfinite(cond[k])) return fail(GMT_EINVAL, "condition value %d is not finite", k);
    TRY(ensure_infer(s, count, st));
    TRY(s->st_cond.upload(cond, 4 * MLP_COND, s->icond.p, st));
    const NetOff o = net_off(1);
    const uint16_t *Wb = (const uint16_t *)s->Pb.p;
    const float *P = (const float *)s->P.p;
    k_cond_bias<<<blocks(64LL * H, 256), 256, 0, st>>>(H, (const unsigned short *)(Wb + o.W1), P + o.b1,
                                                       (const float *)s->icond.p, (float *)s->h0.p);
    k_pack_z<<<blocks((long long)count * 8, 256), 256, 0, st>>>(count, d_eps, (unsigned short *)s->Z8.p);
    HIPCHK(hipGetLastError());
    // first layer over the z columns only: the condition's share is h0
    TRY(gemm(false, true, count, H, 8, (const uint16_t *)s->Z8.p, 8, Wb + o.W1, IN, (const float *)s->h0.p, true,
             nullptr, (uint16_t *)s->A1.p, H, st));
    TRY(gemm(false, true, count, H, H, (const uint16_t *)s->A1.p, H, Wb + o.W2, H, P + o.b2, true, nullptr,
             (uint16_t *)s->A2.p, H, st));
    TRY(gemm(false, true, count, OUT, H, (const uint16_t *)s->A2.p, H, Wb + o.W3, H, P + o.b3, false,
             (float *)s->Dout.p, nullptr, OUT, st));
    return GMT_OK;
}

__global__ void k_first_cols(int count, const float *__restrict__ src, int lds, float *__restrict__ dst) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count * MLP_X) return;
    dst[t] = src[(size_t)(t / MLP_X) * lds + t % MLP_X];
}

}  // namespace

extern "C" gmt_status gmt_sampler_decode(gmt_sampler_t s, const float *cond, const float *d_eps, int32_t count,
                                         float *d_raw, void *stream) {
    if (!d_raw) return fail(GMT_EINVAL, "null output");
    hipStream_t st = (hipStream_t)stream;
    TRY(decode_impl(s, cond, d_eps, count, st));
    k_first_cols<<<blocks((long long)count * MLP_X, 256), 256, 0, st>>>(count, (const float *)s->Dout.p, OUT, d_raw);
    HIPCHK(hipGetLastError());
    return GMT_OK;
}

extern "C" gmt_status gmt_sampler_finish(const float *d_raw, int32_t ldr, int32_t count, const float *boxes,
                                         int32_t m, const float *d_fallback, int32_t ldf, float *d_out, int32_t ld,
                                         int32_t *rejected, void *stream) {
    TRY(check_finish_args(d_raw, ldr, count, d_fallback, ldf, d_out, ld));
    std::vector<int> q;
    TRY(boxes_to_grid(boxes, m, q));
    hipStream_t st = (hipStream_t)stream;
    DevBuf bq, rej;
    gmt_status r = dev_alloc(bq, 4 * q.size(), st);
    if (r == GMT_OK) r = dev_alloc(rej, 4, st);
    // box list and zeroed counter: one synchronous upload of both
    if (r == GMT_OK) {
        q.push_back(0);
        if (hipMemcpyAsync(bq.p, q.data(), 4 * (q.size() - 1), hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(rej.p, &q.back(), 4, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            r = fail(GMT_EDEVICE, "upload of boxes failed");
    }
    if (r == GMT_OK) r = finish_launch(d_raw, ldr, count, (const int *)bq.p, m, d_fallback, ldf, d_out, ld, (int *)rej.p, st);
    if (r == GMT_OK && rejected) {
        if (hipMemcpyAsync(rejected, rej.p, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            r = fail(GMT_EDEVICE, "finish failed");
    }
    dev_free(bq, st);
    dev_free(rej, st);
    return r;
}

extern "C" gmt_status gmt_sampler_generate(gmt_sampler_t s, const float *cond, const float *d_eps, int32_t count,
                                           const float *boxes, int32_t m, const float *d_fallback, int32_t ldf,
                                           float *d_out, int32_t ld, int32_t *rejected, void *stream) {
    if (!s) return fail(GMT_EINVAL, "null sampler");
    std::vector<int> q;
    TRY(boxes_to_grid(boxes, m, q));
    hipStream_t st = (hipStream_t)stream;
    TRY(decode_impl(s, cond, d_eps, count, st));
    TRY(check_finish_args((const float *)s->Dout.p, OUT, count, d_fallback, ldf, d_out, ld));
    q.push_back(0);  // the counter's zero rides along with the boxes
    TRY(s->st_boxes.upload(q.data(), 4 * q.size(), s->boxq.p, st));
    HIPCHK(hipMemcpyAsync(s->rej.p, (const char *)s->boxq.p + 4 * (q.size() - 1), 4, hipMemcpyDeviceToDevice, st));
    TRY(finish_launch((const float *)s->Dout.p, OUT, count, (const int *)s->boxq.p, m, d_fallback, ldf, d_out, ld,
                      (int *)s->rej.p, st));
    if (rejected) {
        HIPCHK(hipMemcpyAsync(rejected, s->rej.p, 4, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    return GMT_OK;
}

extern "C" gmt_status gmt_sampler_destroy(gmt_sampler_t s) {
    if (!s) return GMT_OK;
    if (gmt_host::shut_down()) return GMT_OK;  // left to the process exit
    (void)hipDeviceSynchronize();
    free_train(s);
    free_infer(s);
    for (DevBuf *b : {&s->P, &s->Pb, &s->G, &s->Mo, &s->Vo, &s->cond, &s->targ, &s->owner, &s->boxq, &s->rej})
        dev_free(*b, nullptr);
    s->st_rows.release();
    s->st_cond.release();
    s->st_boxes.release();
    delete s;
    return GMT_OK;
}
