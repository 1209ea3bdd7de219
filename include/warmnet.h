/*
 * warmnet.h -- C ABI of the warm-start network kernels (gfx950).
 *
 * The learned warm start predicts a steady velocity / phase field from the
 * solid mask and the initial phase field; the lattice Boltzmann solver then
 * starts from that prediction and still decides when it has converged.  These
 * entry points are the layers of that network (a 3-D U-Net), written as HIP
 * kernels: 3-D convolutions on BF16 matrix cores (MFMA, FP32 accumulation)
 * over 256-voxel bricks staged with their halo in LDS, their data and weight
 * gradients, pooling, upsampling, channel concatenation, ReLU, the loss and
 * the Adam update.
 *
 * Conventions:
 *   - every tensor pointer is device memory, FP32, channels-last
 *     [n][d][h][w][c]; V = n*d*h*w voxels (a multiple of 16);
 *   - convolution weights are FP32 [c_out][k][k][k][c_in] with k = 1 or 3 and
 *     periodic (circular) padding; the MFMA operands are the inputs rounded
 *     to BF16 (nearest even), accumulation is FP32;
 *   - all work is queued on `stream` (a hipStream_t, NULL = null stream);
 *   - return 0 on success, -1 for invalid arguments, -3 for a HIP error
 *     (wn_last_error() gives the message).
 * The paper has no learned component; this interface exists for the
 * warm-start form of the solver.
 */
#ifndef WARMNET_H
#define WARMNET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* y = conv3d(x, W) + b, then ReLU if relu != 0.  x [V][ci], y [V][co]. */
int wn_conv3d_fwd(const float* x, int n, int d, int h, int w, int ci, const float* W, const float* b, int co,
                  int k, int relu, float* y, void* stream);

/* dx = adjoint of conv3d with respect to x applied to dy.  dy [V][co], dx [V][ci]. */
int wn_conv3d_dgrad(const float* dy, int n, int d, int h, int w, int co, const float* W, int ci, int k, float* dx,
                    void* stream);

/* Workspace bytes needed by wn_conv3d_wgrad for this shape (one FP32 dW per
 * chunk of bricks; the chunk count depends only on the shape); 0 for an
 * invalid shape. */
size_t wn_wgrad_workspace_bytes(int n, int d, int h, int w, int ci, int co, int k);

/* dW = d/dW sum(dy * conv3d(x, W)) (overwrites dW [co][k][k][k][ci]); split
 * over voxel chunks into `workspace` and reduced in a fixed order. */
int wn_conv3d_wgrad(const float* x, const float* dy, int n, int d, int h, int w, int ci, int co, int k, float* dW,
                    void* workspace, size_t workspace_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same weight
 * gradient as wn_conv3d_wgrad, with the chunk partial sums kept in a static
 * device array of wn_wgrad_noalloc_max_bytes() bytes (40 MiB) that the
 * library owns, one copy per GPU, held until the process ends.  Calls no
 * allocating routine.  Returns -1 (and a message) for a shape whose
 * wn_wgrad_workspace_bytes() exceeds that size, -3 for a HIP error.  All
 * calls on one GPU share its array: calls that overlap on one GPU (other
 * streams or host threads) race and must be serialised by the caller. */
size_t wn_wgrad_noalloc_max_bytes(void);
int wn_conv3d_wgrad_noalloc(const float* x, const float* dy, int n, int d, int h, int w, int ci, int co, int k,
                            float* dW, void* stream);

/* Workspace bytes needed by wn_bias_grad for V voxels and co channels. */
size_t wn_bias_grad_workspace_bytes(long long V, int co);

/* db[o] = sum_v dy[v][o] (overwrites), co <= 256; partial sums over blocks of
 * voxels go to `workspace` and are added in a fixed order (deterministic). */
int wn_bias_grad(const float* dy, long long V, int co, float* db, void* workspace, size_t workspace_bytes,
                 void* stream);

/* g[i] = y[i] > 0 ? g[i] : 0, in place. */
int wn_relu_bwd(const float* y, float* g, long long count, void* stream);

/* y[i] += x[i] (gradient accumulation where a tensor feeds two layers). */
int wn_add(const float* x, float* y, long long count, void* stream);

/* y[v][jy] += x[v][jx] for v < V (y has cy channels, x has cx): a residual
 * connection from an input channel to an output channel. */
int wn_add_channel(float* y, int cy, int jy, const float* x, int cx, int jx, long long V, void* stream);

/* 2x2x2 average pooling [n][d][h][w][c] -> [n][d/2][h/2][w/2][c] and its adjoint. */
int wn_pool2_fwd(const float* x, int n, int d, int h, int w, int c, float* y, void* stream);
int wn_pool2_bwd(const float* dy, int n, int d, int h, int w, int c, float* dx, void* stream);

/* nearest 2x upsampling [n][d][h][w][c] -> [n][2d][2h][2w][c] and its adjoint. */
int wn_up2_fwd(const float* x, int n, int d, int h, int w, int c, float* y, void* stream);
int wn_up2_bwd(const float* dy, int n, int d, int h, int w, int c, float* dx, void* stream);

/* y[v] = [a[v] (ca channels), b[v] (cb channels)]; wn_split is its adjoint. */
int wn_concat(const float* a, int ca, const float* b, int cb, long long V, float* y, void* stream);
int wn_split(const float* y, long long V, int ca, int cb, float* a, float* b, void* stream);

/* loss (device, 1 float) = mean((y - t)^2 * wt), grad = d loss / d y, over count
 * values; wt[i % c] weights channel i % c of c channels (NULL: all 1).
 * workspace: device, at least ceil(count / 256) floats (block partials, summed
 * in a fixed order). */
int wn_mse(const float* y, const float* t, const float* wt, int c, long long count, float* loss, float* grad,
           float* workspace, void* stream);

/* One Adam step (Kingma and Ba) on count parameters; step >= 1. */
int wn_adam(float* p, const float* g, float* m, float* v, long long count, float lr, float beta1, float beta2,
            float eps, int step, void* stream);

const char* wn_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* WARMNET_H */
