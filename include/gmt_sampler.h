/* gmt_sampler.h -- learned conditional sampler for the double integrator.
 *
 * The method draws its samples uniformly (Section III-B: Theorem 1 assumes
 * uniform samples); the paper itself has no learning.  This library adds a conditional variational
 * autoencoder that proposes samples concentrated where solution paths of
 * similar queries ran: half of a query's samples come from the network,
 * half stay uniform (and a rejected network sample falls back to a uniform
 * one), so the uniform half keeps the premise of Theorem 1.  The network is
 * trained on waypoints of paths that plain GMT* found.
 *
 * Network (all layers fully connected, FP32 master weights, BF16 inputs and
 * weights on the matrix cores, FP32 accumulation):
 *   encoder  [x(6), 0, 0, c(396), 0 x 12] -> 256 ReLU -> 256 ReLU -> 16
 *            outputs 0..5 mean, 6..11 log variance of q(z | x, c)
 *   decoder  [z(6), 0, 0, c(396), 0 x 12] -> 256 ReLU -> 256 ReLU -> 16
 *            outputs 0..5 the reconstruction of x
 * Condition c (396 floats): x_init (6), goal centre (3), goal radius, 0, 0,
 * then 64 box slots of (lo xyz, hi xyz); unused slots are zero.
 * x is a state in unconstrained coordinates: position p -> logit(p),
 * velocity v -> v / sqrt(1 - |v|^2); gmt_sampler_finish maps back.
 *
 * Parameters: one flat FP32 array, encoder then decoder; per network
 *   W1 [256][416], b1 [256], W2 [256][256], b2 [256], W3 [16][256], b3 [16]
 * (row-major, W[out][in]) -- GMT_SAMPLER_PARAMS floats in all.
 *
 * Loss of a batch of B rows (x, c), with eps ~ N(0, I) supplied per row:
 *   z = mu + exp(lv / 2) eps,
 *   L = mean_b [ w/2 |D(z, c) - x|^2 + beta/2 sum_j (mu_j^2 + exp(lv_j) - 1 - lv_j) ].
 *
 * Device pointers are marked d_; everything else is host memory.  All calls
 * return gmt_status (gmt.h); gmt_last_error() describes failures.  A sampler
 * owns its device buffers: calls on one sampler must not overlap (issue them
 * from one thread, on one stream); different samplers are independent.
 */
#ifndef GMT_SAMPLER_H
#define GMT_SAMPLER_H

#include <stdint.h>

#include "gmt.h"

#ifdef __cplusplus
extern "C" {
#endif

#define GMT_SAMPLER_IN 416
#define GMT_SAMPLER_HIDDEN 256
#define GMT_SAMPLER_OUT 16
#define GMT_SAMPLER_COND 396
#define GMT_SAMPLER_BOX_SLOTS 64
#define GMT_SAMPLER_NET_PARAMS (256 * 416 + 256 + 256 * 256 + 256 + 16 * 256 + 16)
#define GMT_SAMPLER_PARAMS (2 * GMT_SAMPLER_NET_PARAMS)

/* BF16 matrix product on the matrix cores, FP32 accumulation:
 *   C[M][N] = op(A)[M][K] op(B)[K][N] (+ bias[N]) (then max(0, .) if relu)
 * op(A)(m,k) = trans_a ? A[k*lda + m] : A[m*lda + k];
 * op(B)(k,n) = trans_b ? B[n*ldb + k] : B[k*ldb + n].
 * A, B: device BF16 bit patterns, 16-byte aligned; bias: device FP32 or NULL;
 * outputs: C (FP32) and/or Cb (BF16, rounded to nearest even), leading
 * dimension ldc >= N; at least one must be given.  K, lda and ldb must be
 * multiples of 8, as must M when trans_a and N when !trans_b.  M, N, K >= 1.
 * Asynchronous on `stream`. */
gmt_status gmt_gemm_bf16(int32_t trans_a, int32_t trans_b, int32_t M, int32_t N, int32_t K, const uint16_t *d_A,
                         int32_t lda, const uint16_t *d_B, int32_t ldb, const float *d_bias, int32_t relu, float *d_C,
                         uint16_t *d_Cb, int32_t ldc, void *stream);

typedef struct gmt_sampler *gmt_sampler_t;

typedef struct {
    float lr;           /* Adam step size (0 leaves the parameters unchanged) */
    float beta1, beta2; /* Adam moment decays */
    float adam_eps;
    float recon_weight; /* w */
    float kl_weight;    /* beta */
} gmt_train_opts;

/* Create a sampler on the current device with the given FP32 parameters
 * (GMT_SAMPLER_PARAMS floats, copied) and zero Adam moments. */
gmt_status gmt_sampler_create(const float *params, gmt_sampler_t *out);

/* Copy the current FP32 parameters / the gradients of the last training
 * step (GMT_SAMPLER_PARAMS floats each).  Synchronises the sampler. */
gmt_status gmt_sampler_get_params(gmt_sampler_t s, float *params);
gmt_status gmt_sampler_get_grads(gmt_sampler_t s, float *grads);

/* Make a training set resident on the device (replaces any previous one):
 * cond [P][396] conditions, targets [W][6] waypoints in unconstrained
 * coordinates, owner [W] the condition row of each waypoint (0 <= owner < P). */
gmt_status gmt_sampler_set_data(gmt_sampler_t s, const float *cond, int32_t P, const float *targets,
                                const int32_t *owner, int32_t W);

/* One training step on rows[0..B) of the resident set (host indices, each in
 * [0, W)) with d_eps [B][6] standard normal draws: forward, loss, backward,
 * Adam.  B in [8, 65536] and a multiple of 8.  If d_loss is not NULL the
 * batch means of the reconstruction and KL terms are written there (device,
 * 2 floats).  Asynchronous on `stream` except for the copy of `rows`. */
gmt_status gmt_sampler_train_step(gmt_sampler_t s, const int32_t *rows, const float *d_eps, int32_t B,
                                  const gmt_train_opts *opts, float *d_loss, void *stream);

/* Decode `count` samples for one condition (host, 396 floats) from prior
 * draws d_eps [count][6]: d_raw [count][6] receives the raw decoder outputs
 * (unconstrained coordinates).  count in [1, 1 << 24]. */
gmt_status gmt_sampler_decode(gmt_sampler_t s, const float *cond, const float *d_eps, int32_t count, float *d_raw,
                              void *stream);

/* Map raw outputs d_raw [count][ldr] (first 6 values of each row) to states:
 * position sigmoid(u), velocity w / sqrt(1 + |w|^2), each rounded in FP64 to
 * the nearest multiple of 2^-20.  A sample with a non-finite value, with a
 * rounded velocity outside the closed unit ball, or with its position in a
 * closed box of `boxes` (host [m][6] lo xyz, hi xyz, on the grid) is replaced
 * by its fallback d_fallback (SoA [6][ldf]).  Writes SoA d_out [6][ld];
 * *rejected (host, may be NULL) receives the number replaced (then the call
 * synchronises `stream`). */
gmt_status gmt_sampler_finish(const float *d_raw, int32_t ldr, int32_t count, const float *boxes, int32_t m,
                              const float *d_fallback, int32_t ldf, float *d_out, int32_t ld, int32_t *rejected,
                              void *stream);

/* Decode then finish: the learned half of a query's sample set. */
gmt_status gmt_sampler_generate(gmt_sampler_t s, const float *cond, const float *d_eps, int32_t count,
                                const float *boxes, int32_t m, const float *d_fallback, int32_t ldf, float *d_out,
                                int32_t ld, int32_t *rejected, void *stream);

gmt_status gmt_sampler_destroy(gmt_sampler_t s);

#ifdef __cplusplus
}
#endif

#endif /* GMT_SAMPLER_H */
