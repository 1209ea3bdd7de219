// Warm-start network layers on gfx950 (declarations and contract in include/warmnet.h).
//
// 3-D convolutions are implicit GEMMs on the BF16 matrix cores:
//   forward  Y[v][o]  = sum_{k,i} X[v + off_k][i] W[o][k][i]      M = voxels, N = c_out, K = 27 c_in
//   dgrad    dX[v][i] = sum_{k,o} dY[v - off_k][o] W[o][k][i]     M = voxels, N = c_in,  K = 27 c_out
//   wgrad    dW[o][k][i] = sum_v dY[v][o] X[v + off_k][i]         M = c_out,  N = c_in,  K = voxels
// on v_mfma_f32_16x16x16_bf16 (a 16x16 FP32 tile from 16x16 BF16 operands;
// lane l, q = l / 16, r = l % 16, supplies A[r][4q..4q+3] and B[4q..4q+3][r]
// and receives D[4q + j][r], j = 0..3).  A workgroup computes a 64 x 64 output
// tile; each K stage of the operands is rounded to BF16 (nearest even) once
// and staged in LDS, and each of the four wavefronts runs 2 x 2 MFMA tiles on
// it.  Accumulation stays FP32.  The weight gradient splits the voxel sum into
// fixed chunks whose partial tiles are summed in chunk order by a second
// kernel (deterministic).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <string>

#include "warmnet.h"

namespace {

thread_local std::string g_err;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (short)((u >> 16) | ((u & 0x007fffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

struct Grid3 {
    int n, d, h, w;
    __device__ __forceinline__ int shift(int v, int dz, int dy, int dx) const {
        int x = v % w;
        int t = v / w;
        int y = t % h;
        t /= h;
        int z = t % d;
        int b = t / d;
        x += dx;
        x = x < 0 ? x + w : (x >= w ? x - w : x);
        y += dy;
        y = y < 0 ? y + h : (y >= h ? y - h : y);
        z += dz;
        z = z < 0 ? z + d : (z >= d ? z - d : z);
        return ((b * d + z) * h + y) * w + x;
    }
};

__device__ __forceinline__ void koff(int kk, int k, int& dz, int& dy, int& dx) {
    const int r = k / 2;
    dx = kk % k - r;
    dy = (kk / k) % k - r;
    dz = kk / (k * k) - r;
}

// weight gradients split the voxel sum into chunks of this many voxels
constexpr int WG_CHUNK = 4096;

__global__ void __launch_bounds__(256) sum_chunks(const float* __restrict__ part, int nchunk, long long n,
                                                  float* __restrict__ out) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
    for (int c = 0; c < nchunk; ++c) s += part[(size_t)c * n + i];
    out[i] = s;
}

// ---------------------------------------------------------------------------
// LDS-tiled implicit GEMMs (the paths the entry points use).  A workgroup of
// four wavefronts computes a 64 x 64 output tile; per K stage the operands
// (TK wide) are rounded to BF16 once, staged in LDS, and each wavefront runs
// 2 x 2 MFMA 16x16x16 tiles on them (32 x 32 outputs per wavefront).
// LDS rows are padded by 8 BF16 values against bank conflicts.
// ---------------------------------------------------------------------------
constexpr int TM = 64, TN = 64;

template <int TK>
struct Tiles {
    static constexpr int LD = TK + 8;
    short a[TM][LD];
    short b[TN][LD];
};

// the 2 x 2 MFMA tiles of wavefront `wave` on one staged K chunk
template <int TK>
__device__ __forceinline__ void mma_stage(const Tiles<TK>& t, int wave, int q, int r, floatx4 (&acc)[2][2]) {
    const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
#pragma unroll
    for (int ks = 0; ks < TK; ks += 16) {
        bf16x4 af[2], bfr[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) af[i] = *(const bf16x4*)&t.a[wm + i * 16 + r][ks + 4 * q];
#pragma unroll
        for (int j = 0; j < 2; ++j) bfr[j] = *(const bf16x4*)&t.b[wn + j * 16 + r][ks + 4 * q];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[i], bfr[j], acc[i][j], 0, 0, 0);
    }
}

// forward: M = voxels, N = c_out, K = (offset, c_in)
template <int TK>
__global__ void __launch_bounds__(256) conv_fwd_t(const float* __restrict__ X, Grid3 g, int V, int ci,
                                                  const float* __restrict__ W, const float* __restrict__ bias, int co,
                                                  int k, int relu, float* __restrict__ Y) {
    __shared__ Tiles<TK> t;
    constexpr int PER = TK / 4;   // values staged per thread and row (64 rows x TK = 256 threads x PER)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, q = lane >> 4, r = lane & 15;
    const int ntn = (co + TN - 1) / TN;
    const int m0 = (blockIdx.x / ntn) * TM, n0 = (blockIdx.x % ntn) * TN;
    const int K3 = k * k * k;
    const int srow = tid >> 2, scol = (tid & 3) * PER;
    const int sv = m0 + srow, so = n0 + srow;
    floatx4 acc[2][2] = {};
    for (int kk = 0; kk < K3; ++kk) {
        int dz, dy, dx;
        koff(kk, k, dz, dy, dx);
        const int vs = sv < V ? g.shift(sv, dz, dy, dx) : 0;
        for (int c0 = 0; c0 < ci; c0 += TK) {
            short av[PER], bv[PER];
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                const int c = c0 + scol + j;
                av[j] = to_bf16((sv < V && c < ci) ? X[(size_t)vs * ci + c] : 0.f);
                bv[j] = to_bf16((so < co && c < ci) ? W[((size_t)so * K3 + kk) * ci + c] : 0.f);
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                t.a[srow][scol + j] = av[j];
                t.b[srow][scol + j] = bv[j];
            }
            __syncthreads();
            mma_stage<TK>(t, wave, q, r, acc);
        }
    }
    const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int o = n0 + wn + j * 16 + r;
        if (o >= co) continue;
        const float bb = bias ? bias[o] : 0.f;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int v = m0 + wm + i * 16 + 4 * q + e;
                if (v >= V) continue;
                float y = acc[i][j][e] + bb;
                if (relu) y = y > 0.f ? y : 0.f;
                Y[(size_t)v * co + o] = y;
            }
    }
}

// data gradient: M = voxels, N = c_in, K = (offset, c_out)
template <int TK>
__global__ void __launch_bounds__(256) conv_dgrad_t(const float* __restrict__ dY, Grid3 g, int V, int co,
                                                    const float* __restrict__ W, int ci, int k,
                                                    float* __restrict__ dX) {
    __shared__ Tiles<TK> t;
    constexpr int PER = TK / 4;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, q = lane >> 4, r = lane & 15;
    const int ntn = (ci + TN - 1) / TN;
    const int m0 = (blockIdx.x / ntn) * TM, n0 = (blockIdx.x % ntn) * TN;
    const int K3 = k * k * k;
    const int srow = tid >> 2, scol = (tid & 3) * PER;   // A staging: voxel row, c_out columns
    const int sv = m0 + srow;
    // B staging: TK c_out rows of W (contiguous in c_in) -> t.b[c_in][c_out]
    constexpr int BPER = TN * TK / 256;                   // c_in values per thread
    const int bo = tid / (TN / BPER), bi = (tid % (TN / BPER)) * BPER;
    floatx4 acc[2][2] = {};
    for (int kk = 0; kk < K3; ++kk) {
        int dz, dy, dx;
        koff(kk, k, dz, dy, dx);
        const int vs = sv < V ? g.shift(sv, -dz, -dy, -dx) : 0;
        for (int c0 = 0; c0 < co; c0 += TK) {
            short av[PER], bv[BPER];
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                const int o = c0 + scol + j;
                av[j] = to_bf16((sv < V && o < co) ? dY[(size_t)vs * co + o] : 0.f);
            }
            const int o = c0 + bo;
#pragma unroll
            for (int j = 0; j < BPER; ++j) {
                const int i = n0 + bi + j;
                bv[j] = to_bf16((o < co && i < ci) ? W[((size_t)o * K3 + kk) * ci + i] : 0.f);
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < PER; ++j) t.a[srow][scol + j] = av[j];
#pragma unroll
            for (int j = 0; j < BPER; ++j) t.b[bi + j][bo] = bv[j];
            __syncthreads();
            mma_stage<TK>(t, wave, q, r, acc);
        }
    }
    const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int i = n0 + wn + j * 16 + r;
        if (i >= ci) continue;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int v = m0 + wm + a * 16 + 4 * q + e;
                if (v < V) dX[(size_t)v * ci + i] = acc[a][j][e];
            }
    }
}

// weight gradient: M = c_out, N = c_in, K = voxels of one chunk; one offset per
// workgroup; partial[chunk][o][kk][i]
__global__ void __launch_bounds__(256) conv_wgrad_t(const float* __restrict__ X, const float* __restrict__ dY,
                                                    Grid3 g, int V, int ci, int co, int k,
                                                    float* __restrict__ part) {
    constexpr int TK = 32;
    __shared__ Tiles<TK> t;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, q = lane >> 4, r = lane & 15;
    const int K3 = k * k * k;
    const int nmt = (co + TM - 1) / TM, nnt = (ci + TN - 1) / TN;
    int b = blockIdx.x;
    const int mt = b % nmt;
    b /= nmt;
    const int nt = b % nnt;
    b /= nnt;
    const int kk = b % K3;
    const int ch = b / K3;
    const int m0 = mt * TM, n0 = nt * TN;
    int dz, dy, dx;
    koff(kk, k, dz, dy, dx);
    // staging: voxel row tid / 8 (32 voxels per stage), 8 channels at (tid % 8) * 8, written transposed
    const int sv = tid >> 3, sc = (tid & 7) * 8;
    const int vbeg = ch * WG_CHUNK, vend = min(V, vbeg + WG_CHUNK);
    floatx4 acc[2][2] = {};
    for (int v0 = vbeg; v0 < vend; v0 += TK) {
        const int v = v0 + sv;
        const bool ok = v < vend;
        const int vs = ok ? g.shift(v, dz, dy, dx) : 0;
        short av[8], bv[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int o = m0 + sc + j, i = n0 + sc + j;
            av[j] = to_bf16((ok && o < co) ? dY[(size_t)v * co + o] : 0.f);
            bv[j] = to_bf16((ok && i < ci) ? X[(size_t)vs * ci + i] : 0.f);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            t.a[sc + j][sv] = av[j];
            t.b[sc + j][sv] = bv[j];
        }
        __syncthreads();
        mma_stage<TK>(t, wave, q, r, acc);
    }
    const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int i = n0 + wn + j * 16 + r;
        if (i >= ci) continue;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int o = m0 + wm + a * 16 + 4 * q + e;
                if (o < co) part[(((size_t)ch * co + o) * K3 + kk) * ci + i] = acc[a][j][e];
            }
    }
}

// ---------------------------------------------------------------------------
// small layers
// ---------------------------------------------------------------------------
// bias gradient, stage 1: block b sums rows [b * BG_ROWS, ...) of dy [V][co];
// thread t owns column t % co of rows t / co + j * (256 / co), so each pass
// reads a contiguous run of whole rows; partial[b][o] in fixed order
constexpr int BG_ROWS = 512;

__global__ void __launch_bounds__(256) bias_grad_part(const float* __restrict__ dy, long long V, int co,
                                                      float* __restrict__ part) {
    __shared__ float red[256];
    const int t = threadIdx.x;
    const int rpp = 256 / co;                // rows per pass (co <= 256)
    const int o = t % co, r = t / co;
    const long long v0 = (long long)blockIdx.x * BG_ROWS, v1 = min(V, v0 + BG_ROWS);
    float s = 0.f;
    if (r < rpp)
        for (long long v = v0 + r; v < v1; v += rpp) s += dy[v * co + o];
    red[t] = s;
    __syncthreads();
    if (t < co) {
        float acc = 0.f;
        for (int j = 0; j < rpp; ++j) acc += red[j * co + t];
        part[(size_t)blockIdx.x * co + t] = acc;
    }
}

__global__ void __launch_bounds__(256) bias_grad_final(const float* __restrict__ part, int nblk, int co,
                                                       float* __restrict__ db) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= co) return;
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * co + o];
    db[o] = s;
}

__global__ void __launch_bounds__(256) relu_bwd_k(const float* __restrict__ y, float* __restrict__ g, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !(y[i] > 0.f)) g[i] = 0.f;
}

__global__ void __launch_bounds__(256) add_k(const float* __restrict__ x, float* __restrict__ y, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] += x[i];
}

__global__ void __launch_bounds__(256) add_channel_k(float* __restrict__ y, int cy, int jy,
                                                     const float* __restrict__ x, int cx, int jx, long long V) {
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < V) y[v * cy + jy] += x[v * cx + jx];
}

__global__ void __launch_bounds__(256) pool2_fwd_k(const float* __restrict__ x, int n, int d, int h, int w, int c,
                                                   float* __restrict__ y) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int d2 = d / 2, h2 = h / 2, w2 = w / 2;
    const long long tot = (long long)n * d2 * h2 * w2 * c;
    if (i >= tot) return;
    long long t = i;
    const int ch = (int)(t % c);
    t /= c;
    const int xx = (int)(t % w2);
    t /= w2;
    const int yy = (int)(t % h2);
    t /= h2;
    const int zz = (int)(t % d2);
    const int b = (int)(t / d2);
    float s = 0.f;
    for (int a = 0; a < 2; ++a)
        for (int bb = 0; bb < 2; ++bb)
            for (int cc = 0; cc < 2; ++cc)
                s += x[((((size_t)b * d + 2 * zz + a) * h + 2 * yy + bb) * w + 2 * xx + cc) * c + ch];
    y[i] = s * 0.125f;
}

__global__ void __launch_bounds__(256) pool2_bwd_k(const float* __restrict__ dy, int n, int d, int h, int w, int c,
                                                   float* __restrict__ dx) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tot = (long long)n * d * h * w * c;
    if (i >= tot) return;
    long long t = i;
    const int ch = (int)(t % c);
    t /= c;
    const int xx = (int)(t % w);
    t /= w;
    const int yy = (int)(t % h);
    t /= h;
    const int zz = (int)(t % d);
    const int b = (int)(t / d);
    dx[i] = 0.125f * dy[((((size_t)b * (d / 2) + zz / 2) * (h / 2) + yy / 2) * (w / 2) + xx / 2) * c + ch];
}

__global__ void __launch_bounds__(256) up2_fwd_k(const float* __restrict__ x, int n, int d, int h, int w, int c,
                                                 float* __restrict__ y) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int D = 2 * d, Hh = 2 * h, Ww = 2 * w;
    const long long tot = (long long)n * D * Hh * Ww * c;
    if (i >= tot) return;
    long long t = i;
    const int ch = (int)(t % c);
    t /= c;
    const int xx = (int)(t % Ww);
    t /= Ww;
    const int yy = (int)(t % Hh);
    t /= Hh;
    const int zz = (int)(t % D);
    const int b = (int)(t / D);
    y[i] = x[((((size_t)b * d + zz / 2) * h + yy / 2) * w + xx / 2) * c + ch];
}

__global__ void __launch_bounds__(256) up2_bwd_k(const float* __restrict__ dy, int n, int d, int h, int w, int c,
                                                 float* __restrict__ dx) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tot = (long long)n * d * h * w * c;
    if (i >= tot) return;
    long long t = i;
    const int ch = (int)(t % c);
    t /= c;
    const int xx = (int)(t % w);
    t /= w;
    const int yy = (int)(t % h);
    t /= h;
    const int zz = (int)(t % d);
    const int b = (int)(t / d);
    float s = 0.f;
    for (int a = 0; a < 2; ++a)
        for (int bb = 0; bb < 2; ++bb)
            for (int cc = 0; cc < 2; ++cc)
                s += dy[((((size_t)b * 2 * d + 2 * zz + a) * 2 * h + 2 * yy + bb) * 2 * w + 2 * xx + cc) * c + ch];
    dx[i] = s;
}

__global__ void __launch_bounds__(256) concat_k(const float* __restrict__ a, int ca, const float* __restrict__ b,
                                                int cb, long long V, float* __restrict__ y) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = ca + cb;
    if (i >= V * c) return;
    const long long v = i / c;
    const int ch = (int)(i % c);
    y[i] = ch < ca ? a[v * ca + ch] : b[v * cb + ch - ca];
}

__global__ void __launch_bounds__(256) split_k(const float* __restrict__ y, long long V, int ca, int cb,
                                               float* __restrict__ a, float* __restrict__ b) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = ca + cb;
    if (i >= V * c) return;
    const long long v = i / c;
    const int ch = (int)(i % c);
    if (ch < ca) {
        if (a) a[v * ca + ch] = y[i];
    } else if (b) {
        b[v * cb + ch - ca] = y[i];
    }
}

// loss: per-block partial sums then one block in fixed order
__global__ void __launch_bounds__(256) mse_k(const float* __restrict__ y, const float* __restrict__ t,
                                             const float* __restrict__ wt, int c, long long n,
                                             float* __restrict__ grad, float* __restrict__ part) {
    __shared__ float red[256];
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    float s = 0.f;
    if (i < n) {
        const float wi = wt ? wt[i % c] : 1.f;
        const float e = y[i] - t[i];
        s = wi * e * e;
        grad[i] = 2.f * wi * e / (float)n;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) mse_final_k(const float* __restrict__ part, int nb, long long n,
                                                   float* __restrict__ loss) {
    __shared__ float red[256];
    float s = 0.f;
    for (int b = threadIdx.x; b < nb; b += 256) s += part[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = red[0] / (float)n;
}

__global__ void __launch_bounds__(256) adam_k(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, long long n, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

int err(int code, const char* msg) {
    g_err = msg;
    return code;
}

int hip_result(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        g_err = std::string(what) + ": " + hipGetErrorString(e);
        return -3;
    }
    return 0;
}

dim3 blocks_for(long long n) { return dim3((unsigned)((n + 255) / 256)); }

bool shape_ok(int n, int d, int h, int w, int c) {
    if (n < 1 || d < 1 || h < 1 || w < 1 || c < 1) return false;
    const long long V = (long long)n * d * h * w;
    return V % 16 == 0 && V * c < (1LL << 31);
}

}  // namespace

extern "C" {

int wn_conv3d_fwd(const float* x, int n, int d, int h, int w, int ci, const float* W, const float* b, int co, int k,
                  int relu, float* y, void* stream) {
    if (!x || !W || !y || (k != 1 && k != 3) || !shape_ok(n, d, h, w, ci) || co < 1)
        return err(-1, "wn_conv3d_fwd: bad arguments");
    const int V = n * d * h * w;
    const unsigned blocks = (unsigned)(((V + TM - 1) / TM) * ((co + TN - 1) / TN));
    if (ci <= 16)
        hipLaunchKernelGGL(conv_fwd_t<16>, dim3(blocks), dim3(256), 0, (hipStream_t)stream, x, Grid3{n, d, h, w}, V,
                           ci, W, b, co, k, relu, y);
    else
        hipLaunchKernelGGL(conv_fwd_t<32>, dim3(blocks), dim3(256), 0, (hipStream_t)stream, x, Grid3{n, d, h, w}, V,
                           ci, W, b, co, k, relu, y);
    return hip_result("conv_fwd");
}

int wn_conv3d_dgrad(const float* dy, int n, int d, int h, int w, int co, const float* W, int ci, int k, float* dx,
                    void* stream) {
    if (!dy || !W || !dx || (k != 1 && k != 3) || !shape_ok(n, d, h, w, co) || ci < 1)
        return err(-1, "wn_conv3d_dgrad: bad arguments");
    const int V = n * d * h * w;
    const unsigned blocks = (unsigned)(((V + TM - 1) / TM) * ((ci + TN - 1) / TN));
    if (co <= 16)
        hipLaunchKernelGGL(conv_dgrad_t<16>, dim3(blocks), dim3(256), 0, (hipStream_t)stream, dy, Grid3{n, d, h, w},
                           V, co, W, ci, k, dx);
    else
        hipLaunchKernelGGL(conv_dgrad_t<32>, dim3(blocks), dim3(256), 0, (hipStream_t)stream, dy, Grid3{n, d, h, w},
                           V, co, W, ci, k, dx);
    return hip_result("conv_dgrad");
}

size_t wn_wgrad_workspace_bytes(int n, int d, int h, int w, int ci, int co, int k) {
    const long long V = (long long)n * d * h * w;
    const long long nchunk = (V + WG_CHUNK - 1) / WG_CHUNK;
    return (size_t)nchunk * co * k * k * k * ci * sizeof(float);
}

int wn_conv3d_wgrad(const float* x, const float* dy, int n, int d, int h, int w, int ci, int co, int k, float* dW,
                    void* workspace, size_t workspace_bytes, void* stream) {
    if (!x || !dy || !dW || (k != 1 && k != 3) || !shape_ok(n, d, h, w, ci) || co < 1)
        return err(-1, "wn_conv3d_wgrad: bad arguments");
    if (!workspace || workspace_bytes < wn_wgrad_workspace_bytes(n, d, h, w, ci, co, k))
        return err(-1, "wn_conv3d_wgrad: workspace too small");
    const int V = n * d * h * w;
    const int K3 = k * k * k;
    const int nchunk = (V + WG_CHUNK - 1) / WG_CHUNK;
    const long long blocks = (long long)((co + TM - 1) / TM) * ((ci + TN - 1) / TN) * K3 * nchunk;
    hipLaunchKernelGGL(conv_wgrad_t, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, x, dy,
                       Grid3{n, d, h, w}, V, ci, co, k, (float*)workspace);
    const long long nw = (long long)co * K3 * ci;
    hipLaunchKernelGGL(sum_chunks, blocks_for(nw), dim3(256), 0, (hipStream_t)stream, (const float*)workspace,
                       nchunk, nw, dW);
    return hip_result("conv_wgrad");
}

size_t wn_bias_grad_workspace_bytes(long long V, int co) {
    return (size_t)((V + BG_ROWS - 1) / BG_ROWS) * (size_t)(co > 0 ? co : 0) * sizeof(float);
}

int wn_bias_grad(const float* dy, long long V, int co, float* db, void* workspace, size_t workspace_bytes,
                 void* stream) {
    if (!dy || !db || V < 1 || co < 1 || co > 256) return err(-1, "wn_bias_grad: bad arguments");
    if (!workspace || workspace_bytes < wn_bias_grad_workspace_bytes(V, co))
        return err(-1, "wn_bias_grad: workspace too small");
    const int nblk = (int)((V + BG_ROWS - 1) / BG_ROWS);
    hipLaunchKernelGGL(bias_grad_part, dim3(nblk), dim3(256), 0, (hipStream_t)stream, dy, V, co, (float*)workspace);
    hipLaunchKernelGGL(bias_grad_final, dim3((co + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       (const float*)workspace, nblk, co, db);
    return hip_result("bias_grad");
}

int wn_relu_bwd(const float* y, float* g, long long count, void* stream) {
    if (!y || !g || count < 0) return err(-1, "wn_relu_bwd: bad arguments");
    if (count == 0) return 0;
    hipLaunchKernelGGL(relu_bwd_k, blocks_for(count), dim3(256), 0, (hipStream_t)stream, y, g, count);
    return hip_result("relu_bwd");
}

int wn_add(const float* x, float* y, long long count, void* stream) {
    if (!x || !y || count < 0) return err(-1, "wn_add: bad arguments");
    if (count == 0) return 0;
    hipLaunchKernelGGL(add_k, blocks_for(count), dim3(256), 0, (hipStream_t)stream, x, y, count);
    return hip_result("add");
}

int wn_add_channel(float* y, int cy, int jy, const float* x, int cx, int jx, long long V, void* stream) {
    if (!y || !x || cy < 1 || cx < 1 || jy < 0 || jy >= cy || jx < 0 || jx >= cx || V < 0)
        return err(-1, "wn_add_channel: bad arguments");
    if (V == 0) return 0;
    hipLaunchKernelGGL(add_channel_k, blocks_for(V), dim3(256), 0, (hipStream_t)stream, y, cy, jy, x, cx, jx, V);
    return hip_result("add_channel");
}

int wn_pool2_fwd(const float* x, int n, int d, int h, int w, int c, float* y, void* stream) {
    if (!x || !y || n < 1 || c < 1 || d < 2 || h < 2 || w < 2 || (d | h | w) & 1) return err(-1, "wn_pool2_fwd: bad arguments");
    hipLaunchKernelGGL(pool2_fwd_k, blocks_for((long long)n * (d / 2) * (h / 2) * (w / 2) * c), dim3(256), 0,
                       (hipStream_t)stream, x, n, d, h, w, c, y);
    return hip_result("pool2_fwd");
}

int wn_pool2_bwd(const float* dy, int n, int d, int h, int w, int c, float* dx, void* stream) {
    if (!dy || !dx || n < 1 || c < 1 || d < 2 || h < 2 || w < 2 || (d | h | w) & 1) return err(-1, "wn_pool2_bwd: bad arguments");
    hipLaunchKernelGGL(pool2_bwd_k, blocks_for((long long)n * d * h * w * c), dim3(256), 0, (hipStream_t)stream, dy,
                       n, d, h, w, c, dx);
    return hip_result("pool2_bwd");
}

int wn_up2_fwd(const float* x, int n, int d, int h, int w, int c, float* y, void* stream) {
    if (!x || !y || n < 1 || c < 1 || d < 1 || h < 1 || w < 1) return err(-1, "wn_up2_fwd: bad arguments");
    hipLaunchKernelGGL(up2_fwd_k, blocks_for((long long)n * 8 * d * h * w * c), dim3(256), 0, (hipStream_t)stream, x,
                       n, d, h, w, c, y);
    return hip_result("up2_fwd");
}

int wn_up2_bwd(const float* dy, int n, int d, int h, int w, int c, float* dx, void* stream) {
    if (!dy || !dx || n < 1 || c < 1 || d < 1 || h < 1 || w < 1) return err(-1, "wn_up2_bwd: bad arguments");
    hipLaunchKernelGGL(up2_bwd_k, blocks_for((long long)n * d * h * w * c), dim3(256), 0, (hipStream_t)stream, dy, n,
                       d, h, w, c, dx);
    return hip_result("up2_bwd");
}

int wn_concat(const float* a, int ca, const float* b, int cb, long long V, float* y, void* stream) {
    if (!a || !b || !y || ca < 1 || cb < 1 || V < 1) return err(-1, "wn_concat: bad arguments");
    hipLaunchKernelGGL(concat_k, blocks_for(V * (ca + cb)), dim3(256), 0, (hipStream_t)stream, a, ca, b, cb, V, y);
    return hip_result("concat");
}

int wn_split(const float* y, long long V, int ca, int cb, float* a, float* b, void* stream) {
    if (!y || ca < 1 || cb < 1 || V < 1) return err(-1, "wn_split: bad arguments");
    hipLaunchKernelGGL(split_k, blocks_for(V * (ca + cb)), dim3(256), 0, (hipStream_t)stream, y, V, ca, cb, a, b);
    return hip_result("split");
}

int wn_mse(const float* y, const float* t, const float* wt, int c, long long count, float* loss, float* grad,
           float* workspace, void* stream) {
    if (!y || !t || !loss || !grad || !workspace || count < 1 || c < 1) return err(-1, "wn_mse: bad arguments");
    const long long nb = (count + 255) / 256;
    hipLaunchKernelGGL(mse_k, dim3((unsigned)nb), dim3(256), 0, (hipStream_t)stream, y, t, wt, c, count, grad,
                       workspace);
    hipLaunchKernelGGL(mse_final_k, dim3(1), dim3(256), 0, (hipStream_t)stream, (const float*)workspace, (int)nb,
                       count, loss);
    return hip_result("mse");
}

int wn_adam(float* p, const float* g, float* m, float* v, long long count, float lr, float beta1, float beta2,
            float eps, int step, void* stream) {
    if (!p || !g || !m || !v || count < 1 || step < 1) return err(-1, "wn_adam: bad arguments");
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    hipLaunchKernelGGL(adam_k, blocks_for(count), dim3(256), 0, (hipStream_t)stream, p, g, m, v, count, lr, beta1,
                       beta2, eps, c1, c2);
    return hip_result("adam");
}

const char* wn_last_error(void) { return g_err.c_str(); }

}  // extern "C"
