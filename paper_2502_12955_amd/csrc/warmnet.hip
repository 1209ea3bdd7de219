// Warm-start network layers on gfx950 (declarations and contract in include/warmnet.h).
//
// 3-D convolutions with periodic padding on the BF16 matrix cores:
//   forward  Y[v][o]  = sum_{k,i} X[v + off_k][i] W[o][k][i]      M = voxels, N = c_out, K = 27 c_in
//   dgrad    dX[v][i] = sum_{k,o} dY[v - off_k][o] W[o][k][i]     M = voxels, N = c_in,  K = 27 c_out
//   wgrad    dW[o][k][i] = sum_v dY[v][o] X[v + off_k][i]         M = c_out,  N = c_in,  K = voxels
// on v_mfma_f32_16x16x16_bf16 (a 16x16 FP32 tile from 16x16 BF16 operands;
// lane l, q = l / 16, r = l % 16, supplies A[r][4q..4q+3] and B[4q..4q+3][r]
// and receives D[4q + j][r], j = 0..3).  Every operand is rounded to BF16
// (nearest even) once, accumulation stays FP32.  The work is cut into bricks
// of 256 voxels whose input, with its halo, is staged once in LDS (see the
// brick kernels below).  The weight gradient sums over chunks of bricks and
// adds the chunk sums in chunk order in a second kernel (deterministic).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>
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

// the weight gradient's partial sums (one per chunk of bricks) added in a
// fixed order: block b owns 16 outputs; thread (e, c) = (t % 16, t / 16) adds
// chunks c, c + 16, ... of output 16 b + e, then the 16 partials are added
// in order
__global__ void __launch_bounds__(256) sum_chunks(const float* __restrict__ part, int nchunk, long long n,
                                                  float* __restrict__ out) {
    __shared__ float red[16][17];
    const int t = threadIdx.x, e = t & 15, c0 = t >> 4;
    const long long i = (long long)blockIdx.x * 16 + e;
    float s = 0.f;
    if (i < n)
        for (int c = c0; c < nchunk; c += 16) s += part[(size_t)c * n + i];
    red[c0][e] = s;
    __syncthreads();
    if (c0 == 0 && i < n) {
        float a = 0.f;
        for (int j = 0; j < 16; ++j) a += red[j][e];
        out[i] = a;
    }
}

// ---------------------------------------------------------------------------
// Brick convolutions.  The output is cut into bricks of 256 voxels
// (bx x by x bz, chosen per shape; bricks at the far faces may stick out of
// the volume and their outside voxels are neither stored nor summed).  A
// workgroup stages the input around its brick, with the periodic one-voxel
// halo, in LDS as BF16 (rounded once), one chunk of input channels at a time;
// every tap then reads its MFMA operand from LDS at a constant offset, so each
// input value leaves memory once per brick instead of once per tap.
// ---------------------------------------------------------------------------
constexpr int BRICK = 256;
constexpr int MAX_HALO = 600;   // halo voxels of a brick: 48 KB of BF16 staging at 32 channels
constexpr int MAX_XS = 480;     // voxels of a weight-gradient brick's x-shifted input
constexpr int W_LDS = 16384;    // bytes of staged BF16 weights per tap group

struct Brick {
    int bx, by, bz;      // extents, bx * by * bz = BRICK, bx a multiple of 4
    int nbx, nby, nbz;   // bricks per sample along x, y, z
};

// smallest padded volume, then the smallest halo, then the longest x rows
Brick choose_brick(int d, int h, int w) {
    Brick best{};
    long long best_vol = -1;
    int best_halo = 0;
    for (int bx = 32; bx >= 4; bx /= 2)
        for (int by = 1; by <= 16; by *= 2) {
            if (BRICK % (bx * by)) continue;
            const int bz = BRICK / (bx * by);
            if (bz > 16) continue;
            const long long vol = (long long)((d + bz - 1) / bz) * bz * (long long)((h + by - 1) / by) * by *
                                  (long long)((w + bx - 1) / bx) * bx;
            const int halo = (bx + 2) * (by + 2) * (bz + 2);
            if (halo > MAX_HALO || (bz + 2) * (by + 2) * bx > MAX_XS) continue;
            if (best_vol < 0 || vol < best_vol || (vol == best_vol && halo < best_halo)) {
                best = Brick{bx, by, bz, (w + bx - 1) / bx, (h + by - 1) / by, (d + bz - 1) / bz};
                best_vol = vol;
                best_halo = halo;
            }
        }
    return best;
}

// periodic image of a halo coordinate v in [-1, n + 255]: exact for v in
// [-1, n] (every coordinate a voxel inside the volume reads); beyond that
// only voxels outside the volume read it, and it is clamped into range
__device__ __forceinline__ int wrap(int v, int n) {
    v = v < 0 ? v + n : (v >= n ? v - n : v);
    return v < n ? v : n - 1;
}

// blocks are dealt to the eight XCDs round robin; give each XCD a contiguous
// run of logical blocks so that neighbouring bricks share that XCD's L2
__device__ __forceinline__ int xcd_block(int b, int G) {
    const int per = G / 8;
    return b < per * 8 ? (b % 8) * per + b / 8 : b;
}

__device__ __forceinline__ void brick_origin(const Brick& bk, int bi, int& b, int& z0, int& y0, int& x0) {
    x0 = (bi % bk.nbx) * bk.bx;
    bi /= bk.nbx;
    y0 = (bi % bk.nby) * bk.by;
    bi /= bk.nby;
    z0 = (bi % bk.nbz) * bk.bz;
    b = bi / bk.nbz;
}

// Convolution of X [V][C] into Y [V][N] (forward: C = c_in, N = c_out;
// data gradient: X = dY, C = c_out, N = c_in, taps mirrored, W transposed).
// W is the layer's [c_out][K^3][c_in] tensor.  A workgroup computes one brick
// and 16 NR output channels; wavefront `wave` owns brick voxels
// [64 wave, 64 wave + 64) as four MFMA row blocks.  Per chunk of CK input
// channels the halo is staged once and the weights TPG taps at a time, as
// BF16 fragments in MFMA lane order.  Each thread issues all of its staging
// loads before it converts and stores any of them, so a stage costs one
// memory latency; other workgroups on the CU overlap it.  (Prefetching the
// next stage into registers during the matrix work was measured slower: the
// extra registers halve the workgroups per CU.)
template <int K, int CK, int NR>
struct ConvCfg {
    static constexpr int R = K / 2, K3 = K * K * K, LDA = CK + 8, C4 = CK / 4, KS = CK / 16;
    static constexpr int TPG = K == 1                          ? 1
                               : 27 * KS * NR * 64 * 8 <= W_LDS ? 27
                               : 9 * KS * NR * 64 * 8 <= W_LDS  ? 9
                                                                : 3;
    static constexpr int NG = K3 / TPG;
    static constexpr int WITEMS = TPG * KS * NR * 64;                 // bf16x4 fragments per group
    static constexpr int WPT = (WITEMS + 255) / 256;                  // per thread
    static constexpr int HMAX = K == 1 ? BRICK : MAX_HALO;
    static constexpr int HPT = (HMAX * C4 + 255) / 256;               // halo float4 per thread
    static constexpr size_t lds_bytes = (size_t)HMAX * LDA * 2 + (size_t)WITEMS * 8;
};

template <int K, int CK, int NR, bool DGRAD>
__global__ void __launch_bounds__(256) conv_brick(const float* __restrict__ X, int C, Grid3 g, Brick bk,
                                                  const float* __restrict__ W, const float* __restrict__ bias,
                                                  int N, int relu, float* __restrict__ Y) {
    constexpr bool dgrad = DGRAD;
    using F = ConvCfg<K, CK, NR>;
    static_assert(F::lds_bytes <= 65536 && F::WITEMS * 8 <= W_LDS, "conv_brick staging exceeds 64 KiB of LDS");
    constexpr int R = F::R, K3 = F::K3, LDA = F::LDA, C4 = F::C4, KS = F::KS, TPG = F::TPG, NG = F::NG;
    extern __shared__ short lds[];
    short* halo = lds;                                   // [HV][LDA]
    bf16x4* wl = (bf16x4*)(lds + F::HMAX * LDA);         // [TPG][KS][NR][64]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, q = lane >> 4, r = lane & 15;
    const int ntn = (N + 16 * NR - 1) / (16 * NR);
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int n0 = (lb % ntn) * 16 * NR;
    int b, z0, y0, x0;
    brick_origin(bk, lb / ntn, b, z0, y0, x0);
    const int HX = bk.bx + 2 * R, HY = bk.by + 2 * R, HV = HX * HY * (bk.bz + 2 * R);
    const bool vec = (C & 3) == 0;

    float4 hreg[F::HPT];
    auto load_halo = [&](int c0) {
#pragma unroll
        for (int j = 0; j < F::HPT; ++j) {
            const int it = tid + 256 * j;
            float4 t = make_float4(0.f, 0.f, 0.f, 0.f);
            if (it < HV * C4) {
                const int hv = it / C4, c = c0 + (it % C4) * 4;
                const int hx = hv % HX, hy = (hv / HX) % HY, hz = hv / (HX * HY);
                const long long vox =
                    ((long long)(b * g.d + wrap(z0 + hz - R, g.d)) * g.h + wrap(y0 + hy - R, g.h)) * g.w +
                    wrap(x0 + hx - R, g.w);
                const float* src = X + vox * C + c;
                if (vec && c + 3 < C) {
                    t = *(const float4*)src;
                } else {
                    t.x = c < C ? src[0] : 0.f;
                    t.y = c + 1 < C ? src[1] : 0.f;
                    t.z = c + 2 < C ? src[2] : 0.f;
                    t.w = c + 3 < C ? src[3] : 0.f;
                }
            }
            hreg[j] = t;
        }
    };
    auto store_halo = [&]() {
#pragma unroll
        for (int j = 0; j < F::HPT; ++j) {
            const int it = tid + 256 * j;
            if (it < HV * C4) {
                bf16x4 o;
                o[0] = to_bf16(hreg[j].x), o[1] = to_bf16(hreg[j].y), o[2] = to_bf16(hreg[j].z),
                o[3] = to_bf16(hreg[j].w);
                *(bf16x4*)&halo[(it / C4) * LDA + (it % C4) * 4] = o;
            }
        }
    };
    float4 wreg[F::WPT];
    // Weight fragments: lane (q, r) of fragment (tt, ks, nb) holds
    // B[4q + j][r] = W'(c = c0 + 16 ks + 4q + j, n = n0 + 16 nb + r) of tap
    // grp TPG + tt.  Item `it` loads four values contiguous in W: along c for
    // the forward pass (fragment `it`, lane it % 64), along n for the data
    // gradient (fragment it / 64, c offset (it % 64) / 4, lanes r = 4 ((it % 64) % 4) + j).
    const bool wvec = DGRAD ? (N & 3) == 0 : (C & 3) == 0;
    auto load_w = [&](int c0, int grp) {
#pragma unroll
        for (int j = 0; j < F::WPT; ++j) {
            const int it = tid + 256 * j;
            float4 t = make_float4(0.f, 0.f, 0.f, 0.f);
            if (it < F::WITEMS) {
                const int l = it & 63, nb = (it >> 6) % NR, ks = (it >> 6) / NR % KS, tt = (it >> 6) / NR / KS;
                const int kk = grp * TPG + tt;
                if constexpr (!dgrad) {
                    const int n = n0 + nb * 16 + (l & 15), c = c0 + ks * 16 + 4 * (l >> 4);
                    const float* src = W + ((size_t)n * K3 + kk) * C + c;
                    if (n < N) {
                        if (wvec && c + 3 < C) {
                            t = *(const float4*)src;
                        } else {
                            t.x = c < C ? src[0] : 0.f;
                            t.y = c + 1 < C ? src[1] : 0.f;
                            t.z = c + 2 < C ? src[2] : 0.f;
                            t.w = c + 3 < C ? src[3] : 0.f;
                        }
                    }
                } else {
                    const int c = c0 + ks * 16 + (l >> 2), n = n0 + nb * 16 + 4 * (l & 3);
                    const float* src = W + ((size_t)c * K3 + (K3 - 1 - kk)) * N + n;
                    if (c < C) {
                        if (wvec && n + 3 < N) {
                            t = *(const float4*)src;
                        } else {
                            t.x = n < N ? src[0] : 0.f;
                            t.y = n + 1 < N ? src[1] : 0.f;
                            t.z = n + 2 < N ? src[2] : 0.f;
                            t.w = n + 3 < N ? src[3] : 0.f;
                        }
                    }
                }
            }
            wreg[j] = t;
        }
    };
    auto store_w = [&]() {
#pragma unroll
        for (int j = 0; j < F::WPT; ++j) {
            const int it = tid + 256 * j;
            if (it < F::WITEMS) {
                if constexpr (!dgrad) {
                    bf16x4 o;
                    o[0] = to_bf16(wreg[j].x), o[1] = to_bf16(wreg[j].y), o[2] = to_bf16(wreg[j].z),
                    o[3] = to_bf16(wreg[j].w);
                    wl[it] = o;
                } else {
                    // c offset cc = (it % 64) / 4 -> q = cc / 4, element cc % 4; r = 4 (it % 4) + jj
                    const int l = it & 63, cc = l >> 2;
                    short* frag = (short*)&wl[it & ~63];
                    const int e = cc & 3, lb = (cc >> 2) * 16 + 4 * (l & 3);
                    frag[(lb + 0) * 4 + e] = to_bf16(wreg[j].x);
                    frag[(lb + 1) * 4 + e] = to_bf16(wreg[j].y);
                    frag[(lb + 2) * 4 + e] = to_bf16(wreg[j].z);
                    frag[(lb + 3) * 4 + e] = to_bf16(wreg[j].w);
                }
            }
        }
    };

    int hv0[4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
        const int m = wave * 64 + mb * 16 + r;
        const int mx = m % bk.bx, my = (m / bk.bx) % bk.by, mz = m / (bk.bx * bk.by);
        hv0[mb] = ((mz + R) * HY + my + R) * HX + mx + R;
    }
    floatx4 acc[4][NR] = {};
    for (int c0 = 0; c0 < C; c0 += CK) {
        for (int grp = 0; grp < NG; ++grp) {
            if (grp == 0) load_halo(c0);
            load_w(c0, grp);
            __syncthreads();
            if (grp == 0) store_halo();
            store_w();
            __syncthreads();
#pragma unroll 1
            for (int tt = 0; tt < TPG; ++tt) {
                int dz, dy, dx;
                koff(grp * TPG + tt, K, dz, dy, dx);
                const int toff = (dz * HY + dy) * HX + dx;
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    bf16x4 bf[NR];
#pragma unroll
                    for (int nb = 0; nb < NR; ++nb) bf[nb] = wl[((tt * KS + ks) * NR + nb) * 64 + lane];
#pragma unroll
                    for (int mb = 0; mb < 4; ++mb) {
                        const bf16x4 af = *(const bf16x4*)&halo[(hv0[mb] + toff) * LDA + ks * 16 + 4 * q];
#pragma unroll
                        for (int nb = 0; nb < NR; ++nb)
                            acc[mb][nb] =
                                __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af, bf[nb], acc[mb][nb], 0, 0, 0);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int nb = 0; nb < NR; ++nb) {
        const int n = n0 + nb * 16 + r;
        if (n >= N) continue;
        const float bb = bias ? bias[n] : 0.f;
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int m = wave * 64 + mb * 16 + 4 * q + j;
                const int x = x0 + m % bk.bx, y = y0 + (m / bk.bx) % bk.by, z = z0 + m / (bk.bx * bk.by);
                if (x >= g.w || y >= g.h || z >= g.d) continue;
                float val = acc[mb][nb][j] + bb;
                if (relu) val = val > 0.f ? val : 0.f;
                Y[(((long long)(b * g.d + z) * g.h + y) * g.w + x) * N + n] = val;
            }
    }
}

// Weight gradient dW[o][tap][i] = sum_v dY[v][o] X[v + off(tap)][i].
// MFMA M = output channels (16 MO per workgroup), N = input channels (16 NI),
// K = voxels of a brick, in groups of four along x.  A workgroup owns one x
// offset dx of the taps (the nine (dz, dy) taps sharing it), so the input is
// staged with that x shift applied and every operand read stays aligned.
// Wavefront `wave` takes the voxel groups 16 (wave + 4 j) of every brick.
// The four wavefronts' sums are added in LDS in wavefront order and the
// chunk's sum goes to part[chunk][o][tap][i].
template <int K, int MO, int NI>
struct WgradCfg {
    static constexpr int R = K / 2, K3 = K * K * K, T = K == 3 ? 9 : 1, NDX = K == 3 ? 3 : 1;
    static constexpr int LDY = BRICK + 4;
    static constexpr int XMAX = K == 1 ? BRICK : MAX_XS;
    static constexpr int YPT = BRICK * 4 * MO / 256;                  // dY float4 per thread
    static constexpr int XPT = (XMAX * 4 * NI + 255) / 256;           // X float4 per thread
    static constexpr size_t stage_bytes = ((size_t)16 * MO * LDY + (size_t)16 * NI * (XMAX + 4)) * 2;
    static constexpr size_t red_bytes = (size_t)T * MO * NI * 256 * 4;
    static constexpr size_t lds_bytes = stage_bytes > red_bytes ? stage_bytes : red_bytes;
};

template <int K, int MO, int NI>
__global__ void __launch_bounds__(256) wgrad_brick(const float* __restrict__ X, int ci,
                                                   const float* __restrict__ dY, int co, Grid3 g, Brick bk,
                                                   int bricks_per_chunk, int nbricks, float* __restrict__ part) {
    using F = WgradCfg<K, MO, NI>;
    static_assert(F::lds_bytes <= 65536, "wgrad_brick staging exceeds 64 KiB of LDS");
    constexpr int R = F::R, K3 = F::K3, T = F::T, NDX = F::NDX, LDY = F::LDY;
    extern __shared__ short lds[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, q = lane >> 4, r = lane & 15;
    const int nci = (ci + 16 * NI - 1) / (16 * NI), nco = (co + 16 * MO - 1) / (16 * MO);
    int lb = xcd_block(blockIdx.x, gridDim.x);
    const int cot = lb % nco;
    lb /= nco;
    const int cit = lb % nci;
    lb /= nci;
    const int dx = lb % NDX - R;
    const int chunk = lb / NDX;
    const int o0 = cot * 16 * MO, i0 = cit * 16 * NI;
    const int HY = bk.by + 2 * R, XS = (bk.bz + 2 * R) * HY * bk.bx, LDX = XS + 4;
    short* dyt = lds;                       // [16 MO][LDY]
    short* xs = lds + 16 * MO * LDY;        // [16 NI][LDX]
    const bool vy = (co & 3) == 0, vx = (ci & 3) == 0;

    float4 yreg[F::YPT], xreg[F::XPT];
    auto load_brick = [&](int bi) {
        int b, z0, y0, x0;
        brick_origin(bk, bi, b, z0, y0, x0);
#pragma unroll
        for (int j = 0; j < F::YPT; ++j) {
            const int it = tid + 256 * j;
            const int m = it / (4 * MO), o = o0 + 4 * (it % (4 * MO));
            const int x = x0 + m % bk.bx, y = y0 + (m / bk.bx) % bk.by, z = z0 + m / (bk.bx * bk.by);
            float4 t = make_float4(0.f, 0.f, 0.f, 0.f);
            if (x < g.w && y < g.h && z < g.d) {
                const float* src = dY + (((long long)(b * g.d + z) * g.h + y) * g.w + x) * co + o;
                if (vy && o + 3 < co) {
                    t = *(const float4*)src;
                } else {
                    t.x = o < co ? src[0] : 0.f;
                    t.y = o + 1 < co ? src[1] : 0.f;
                    t.z = o + 2 < co ? src[2] : 0.f;
                    t.w = o + 3 < co ? src[3] : 0.f;
                }
            }
            yreg[j] = t;
        }
#pragma unroll
        for (int j = 0; j < F::XPT; ++j) {
            const int it = tid + 256 * j;
            float4 t = make_float4(0.f, 0.f, 0.f, 0.f);
            if (it < XS * 4 * NI) {
                const int p = it / (4 * NI), i = i0 + 4 * (it % (4 * NI));
                const int px = p % bk.bx, py = (p / bk.bx) % HY, pz = p / (bk.bx * HY);
                const long long vox =
                    ((long long)(b * g.d + wrap(z0 + pz - R, g.d)) * g.h + wrap(y0 + py - R, g.h)) * g.w +
                    wrap(x0 + px + dx, g.w);
                const float* src = X + vox * ci + i;
                if (vx && i + 3 < ci) {
                    t = *(const float4*)src;
                } else {
                    t.x = i < ci ? src[0] : 0.f;
                    t.y = i + 1 < ci ? src[1] : 0.f;
                    t.z = i + 2 < ci ? src[2] : 0.f;
                    t.w = i + 3 < ci ? src[3] : 0.f;
                }
            }
            xreg[j] = t;
        }
    };
    auto store_brick = [&]() {
#pragma unroll
        for (int j = 0; j < F::YPT; ++j) {
            const int it = tid + 256 * j;
            const int m = it / (4 * MO), o = 4 * (it % (4 * MO));
            dyt[(o + 0) * LDY + m] = to_bf16(yreg[j].x);
            dyt[(o + 1) * LDY + m] = to_bf16(yreg[j].y);
            dyt[(o + 2) * LDY + m] = to_bf16(yreg[j].z);
            dyt[(o + 3) * LDY + m] = to_bf16(yreg[j].w);
        }
#pragma unroll
        for (int j = 0; j < F::XPT; ++j) {
            const int it = tid + 256 * j;
            if (it < XS * 4 * NI) {
                const int p = it / (4 * NI), i = 4 * (it % (4 * NI));
                xs[(i + 0) * LDX + p] = to_bf16(xreg[j].x);
                xs[(i + 1) * LDX + p] = to_bf16(xreg[j].y);
                xs[(i + 2) * LDX + p] = to_bf16(xreg[j].z);
                xs[(i + 3) * LDX + p] = to_bf16(xreg[j].w);
            }
        }
    };

    floatx4 acc[T][MO][NI] = {};
    const int bbeg = chunk * bricks_per_chunk, bend = min(nbricks, bbeg + bricks_per_chunk);
    for (int bi = bbeg; bi < bend; ++bi) {
        load_brick(bi);
        __syncthreads();
        store_brick();
        __syncthreads();
#pragma unroll 1
        for (int kq = wave; kq < BRICK / 16; kq += 4) {
            const int m = kq * 16 + 4 * q;   // first of this lane's four voxels (one x row)
            const int mx = m % bk.bx, my = (m / bk.bx) % bk.by, mz = m / (bk.bx * bk.by);
            bf16x4 af[MO];
#pragma unroll
            for (int mo = 0; mo < MO; ++mo) af[mo] = *(const bf16x4*)&dyt[(mo * 16 + r) * LDY + m];
#pragma unroll
            for (int t = 0; t < T; ++t) {
                const int dz = K == 3 ? t / 3 - 1 : 0, dy = K == 3 ? t % 3 - 1 : 0;
                const int p = ((mz + dz + R) * HY + my + dy + R) * bk.bx + mx;
#pragma unroll
                for (int ni = 0; ni < NI; ++ni) {
                    const bf16x4 bfr = *(const bf16x4*)&xs[(ni * 16 + r) * LDX + p];
#pragma unroll
                    for (int mo = 0; mo < MO; ++mo)
                        acc[t][mo][ni] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[mo], bfr, acc[t][mo][ni], 0, 0, 0);
                }
            }
        }
    }
    // add the four wavefronts' sums in wavefront order
    float* red = (float*)lds;
    for (int w = 0; w < 4; ++w) {
        __syncthreads();
        if (wave == w) {
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int mo = 0; mo < MO; ++mo)
#pragma unroll
                    for (int ni = 0; ni < NI; ++ni) {
                        float* dst = red + ((t * MO + mo) * NI + ni) * 256 + lane * 4;
#pragma unroll
                        for (int j = 0; j < 4; ++j) dst[j] = w == 0 ? acc[t][mo][ni][j] : dst[j] + acc[t][mo][ni][j];
                    }
        }
    }
    __syncthreads();
    for (int e = tid; e < T * MO * NI * 256; e += 256) {
        const int tile = e / 256, l = (e % 256) / 4, j = e % 4;
        const int ni = tile % NI, mo = (tile / NI) % MO, t = tile / (NI * MO);
        const int o = o0 + mo * 16 + 4 * (l >> 4) + j, i = i0 + ni * 16 + (l & 15);
        if (o >= co || i >= ci) continue;
        const int kk = K == 3 ? t * 3 + dx + 1 : 0;
        part[(((size_t)chunk * co + o) * K3 + kk) * ci + i] = red[e];
    }
}

// ---------------------------------------------------------------------------
// small layers
// ---------------------------------------------------------------------------
// bias gradient, stage 1: thread t owns column t % co (co <= 256) and every
// (256 / co)-th row from t / co on, BG_PER rows in all (independent loads);
// the block's BG_PER * (256 / co) rows are summed in LDS in a fixed order
// into part[block][o]
constexpr int BG_PER = 16;

__host__ __device__ inline long long bg_rows(int co) { return (long long)BG_PER * (256 / co); }

__global__ void __launch_bounds__(256) bias_grad_part(const float* __restrict__ dy, long long V, int co,
                                                      float* __restrict__ part) {
    __shared__ float red[256];
    const int t = threadIdx.x;
    const int rpp = 256 / co;
    const int o = t % co, r = t / co;
    const long long v0 = (long long)blockIdx.x * bg_rows(co);
    float s = 0.f;
    if (r < rpp) {
        float v[BG_PER];
#pragma unroll
        for (int j = 0; j < BG_PER; ++j) {
            const long long row = v0 + r + (long long)j * rpp;
            v[j] = row < V ? dy[row * co + o] : 0.f;
        }
#pragma unroll
        for (int j = 0; j < BG_PER; ++j) s += v[j];
    }
    red[t] = s;
    __syncthreads();
    if (t < co) {
        float acc = 0.f;
        for (int j = 0; j < rpp; ++j) acc += red[j * co + t];
        part[(size_t)blockIdx.x * co + t] = acc;
    }
}

// stage 2: block o adds part[.][o] (strided per thread, then a fixed tree)
__global__ void __launch_bounds__(256) bias_grad_final(const float* __restrict__ part, int nblk, int co,
                                                       float* __restrict__ db) {
    __shared__ float red[256];
    const int o = blockIdx.x, t = threadIdx.x;
    float s = 0.f;
    for (int b = t; b < nblk; b += 256) s += part[(size_t)b * co + o];
    red[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) db[o] = red[0];
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

// ---- convolution launch plans --------------------------------------------
template <int K, int CK, int NR>
void conv_go(const float* X, int C, Grid3 g, Brick bk, const float* W, int dgrad, const float* bias, int N, int relu,
             float* Y, int blocks, hipStream_t st) {
    const size_t bytes = ConvCfg<K, CK, NR>::lds_bytes;
    if (dgrad)
        hipLaunchKernelGGL((conv_brick<K, CK, NR, true>), dim3(blocks), dim3(256), bytes, st, X, C, g, bk, W, bias, N,
                           relu, Y);
    else
        hipLaunchKernelGGL((conv_brick<K, CK, NR, false>), dim3(blocks), dim3(256), bytes, st, X, C, g, bk, W, bias, N,
                           relu, Y);
}

template <int K, int CK>
void conv_nr(int NR, const float* X, int C, Grid3 g, Brick bk, const float* W, int dgrad, const float* bias, int N,
             int relu, float* Y, int blocks, hipStream_t st) {
    switch (NR) {
        case 1: conv_go<K, CK, 1>(X, C, g, bk, W, dgrad, bias, N, relu, Y, blocks, st); break;
        case 2: conv_go<K, CK, 2>(X, C, g, bk, W, dgrad, bias, N, relu, Y, blocks, st); break;
        case 3: conv_go<K, CK, 3>(X, C, g, bk, W, dgrad, bias, N, relu, Y, blocks, st); break;
        default: conv_go<K, CK, 4>(X, C, g, bk, W, dgrad, bias, N, relu, Y, blocks, st); break;
    }
}

// channel chunk: 32 unless that pads C further than 16 does; output tile:
// up to 64 channels, split into 16-channel tiles when the bricks alone leave
// the chip with too few workgroups
void launch_conv(const float* X, int C, Grid3 g, const float* W, int dgrad, const float* bias, int N, int k, int relu,
                 float* Y, hipStream_t st) {
    const Brick bk = choose_brick(g.d, g.h, g.w);
    const int nbricks = g.n * bk.nbx * bk.nby * bk.nbz;
    const int nb16 = (N + 15) / 16;
    int ntile = (nb16 + 3) / 4;
    int NR = (nb16 + ntile - 1) / ntile;
    if (nbricks * ntile < 1024) {
        NR = 1;
        ntile = nb16;
    }
    const int blocks = nbricks * ntile;
    const bool ck32 = (C + 31) / 32 * 32 == (C + 15) / 16 * 16;
    if (k == 3) {
        if (ck32) conv_nr<3, 32>(NR, X, C, g, bk, W, dgrad, bias, N, relu, Y, blocks, st);
        else conv_nr<3, 16>(NR, X, C, g, bk, W, dgrad, bias, N, relu, Y, blocks, st);
    } else {
        if (ck32) conv_nr<1, 32>(NR, X, C, g, bk, W, dgrad, bias, N, relu, Y, blocks, st);
        else conv_nr<1, 16>(NR, X, C, g, bk, W, dgrad, bias, N, relu, Y, blocks, st);
    }
}

struct WgradPlan {
    Brick bk;
    int MO, NI, nbricks, bricks_per_chunk, nchunk, blocks;
};

// output-channel tile 16 MO (MO in 1, 2, 4) and input-channel chunk 16 NI
// (NI in 1, 2; 1 when MO = 4), the one padding c_in least; about a thousand
// workgroups, each summing a run of consecutive bricks
WgradPlan wgrad_plan(int n, int d, int h, int w, int ci, int co, int k) {
    WgradPlan p;
    p.bk = choose_brick(d, h, w);
    p.nbricks = n * p.bk.nbx * p.bk.nby * p.bk.nbz;
    const int cb = (co + 15) / 16;
    p.MO = cb == 1 ? 1 : cb == 2 ? 2 : 4;
    p.NI = 1;
    if (p.MO < 4 && (ci + 31) / 32 * 32 == (ci + 15) / 16 * 16) p.NI = 2;
    const int nci = (ci + 16 * p.NI - 1) / (16 * p.NI), nco = (co + 16 * p.MO - 1) / (16 * p.MO);
    const int per = (k == 3 ? 3 : 1) * nci * nco;
    const int target = std::max(1, 1024 / per);
    p.bricks_per_chunk = (p.nbricks + target - 1) / target;
    p.nchunk = (p.nbricks + p.bricks_per_chunk - 1) / p.bricks_per_chunk;
    p.blocks = p.nchunk * per;
    return p;
}

template <int K, int MO, int NI>
void wgrad_go(const WgradPlan& pl, const float* X, int ci, const float* dY, int co, Grid3 g, float* part,
              hipStream_t st) {
    const size_t bytes = WgradCfg<K, MO, NI>::lds_bytes;
    hipLaunchKernelGGL((wgrad_brick<K, MO, NI>), dim3(pl.blocks), dim3(256), bytes, st, X, ci, dY, co, g, pl.bk,
                       pl.bricks_per_chunk, pl.nbricks, part);
}

template <int K>
void wgrad_k(const WgradPlan& pl, const float* X, int ci, const float* dY, int co, Grid3 g, float* part,
             hipStream_t st) {
    if (pl.MO == 1 && pl.NI == 1) wgrad_go<K, 1, 1>(pl, X, ci, dY, co, g, part, st);
    else if (pl.MO == 1) wgrad_go<K, 1, 2>(pl, X, ci, dY, co, g, part, st);
    else if (pl.MO == 2 && pl.NI == 1) wgrad_go<K, 2, 1>(pl, X, ci, dY, co, g, part, st);
    else if (pl.MO == 2) wgrad_go<K, 2, 2>(pl, X, ci, dY, co, g, part, st);
    else wgrad_go<K, 4, 1>(pl, X, ci, dY, co, g, part, st);
}

void launch_wgrad(const WgradPlan& pl, const float* X, int ci, const float* dY, int co, Grid3 g, int k, float* part,
                  hipStream_t st) {
    if (k == 3) wgrad_k<3>(pl, X, ci, dY, co, g, part, st);
    else wgrad_k<1>(pl, X, ci, dY, co, g, part, st);
}

}  // namespace

extern "C" {

int wn_conv3d_fwd(const float* x, int n, int d, int h, int w, int ci, const float* W, const float* b, int co, int k,
                  int relu, float* y, void* stream) {
    if (!x || !W || !y || (k != 1 && k != 3) || !shape_ok(n, d, h, w, ci) || !shape_ok(n, d, h, w, co))
        return err(-1, "wn_conv3d_fwd: bad arguments");
    launch_conv(x, ci, Grid3{n, d, h, w}, W, 0, b, co, k, relu, y, (hipStream_t)stream);
    return hip_result("conv_fwd");
}

int wn_conv3d_dgrad(const float* dy, int n, int d, int h, int w, int co, const float* W, int ci, int k, float* dx,
                    void* stream) {
    if (!dy || !W || !dx || (k != 1 && k != 3) || !shape_ok(n, d, h, w, co) || !shape_ok(n, d, h, w, ci))
        return err(-1, "wn_conv3d_dgrad: bad arguments");
    launch_conv(dy, co, Grid3{n, d, h, w}, W, 1, nullptr, ci, k, 0, dx, (hipStream_t)stream);
    return hip_result("conv_dgrad");
}

size_t wn_wgrad_workspace_bytes(int n, int d, int h, int w, int ci, int co, int k) {
    if (n < 1 || d < 1 || h < 1 || w < 1 || ci < 1 || co < 1 || (k != 1 && k != 3)) return 0;
    const WgradPlan pl = wgrad_plan(n, d, h, w, ci, co, k);
    return (size_t)pl.nchunk * co * k * k * k * ci * sizeof(float);
}

int wn_conv3d_wgrad(const float* x, const float* dy, int n, int d, int h, int w, int ci, int co, int k, float* dW,
                    void* workspace, size_t workspace_bytes, void* stream) {
    if (!x || !dy || !dW || (k != 1 && k != 3) || !shape_ok(n, d, h, w, ci) || !shape_ok(n, d, h, w, co))
        return err(-1, "wn_conv3d_wgrad: bad arguments");
    if (!workspace || workspace_bytes < wn_wgrad_workspace_bytes(n, d, h, w, ci, co, k))
        return err(-1, "wn_conv3d_wgrad: workspace too small");
    const WgradPlan pl = wgrad_plan(n, d, h, w, ci, co, k);
    launch_wgrad(pl, x, ci, dy, co, Grid3{n, d, h, w}, k, (float*)workspace, (hipStream_t)stream);
    const long long nw = (long long)co * k * k * k * ci;
    hipLaunchKernelGGL(sum_chunks, dim3((unsigned)((nw + 15) / 16)), dim3(256), 0, (hipStream_t)stream,
                       (const float*)workspace, pl.nchunk, nw, dW);
    return hip_result("conv_wgrad");
}

// ---------------------------------------------------------------------------
// no-allocation weight gradient: the chunk partial sums live in a file-scope
// device array instead of a caller workspace.  Each GPU holds its own copy of
// the array; its device address is looked up once per device on the first
// call made with that device current and kept in scratch_ptr[].  Every call on
// one GPU reuses that GPU's array, so calls that overlap on one GPU (other
// streams or threads) race on it.  Every partial that sum_chunks reads is
// written first by the same call, so nothing needs clearing.
// ---------------------------------------------------------------------------
}  // extern "C"
namespace {
constexpr size_t kScratchBytes = (size_t)40 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) float scratch[kScratchBytes / sizeof(float)];
void* scratch_ptr[kMaxDevices];
std::mutex scratch_mu;

int scratch_for_current_device(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return err(-3, (std::string("hipGetDevice: ") + hipGetErrorString(e)).c_str());
    if (dev < 0 || dev >= kMaxDevices) return err(-1, "wn_conv3d_wgrad_noalloc: device ordinal out of range");
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return err(-3, (std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)).c_str());
        scratch_ptr[dev] = p;
    }
    *out = scratch_ptr[dev];
    return 0;
}
}  // namespace
extern "C" {

size_t wn_wgrad_noalloc_max_bytes(void) { return kScratchBytes; }

int wn_conv3d_wgrad_noalloc(const float* x, const float* dy, int n, int d, int h, int w, int ci, int co, int k,
                            float* dW, void* stream) {
    if (!x || !dy || !dW || (k != 1 && k != 3) || !shape_ok(n, d, h, w, ci) || !shape_ok(n, d, h, w, co))
        return err(-1, "wn_conv3d_wgrad_noalloc: bad arguments");
    const size_t need = wn_wgrad_workspace_bytes(n, d, h, w, ci, co, k);
    if (need > kScratchBytes)
        return err(-1, ("wn_conv3d_wgrad_noalloc: this shape needs " + std::to_string(need) +
                        " bytes of partial sums, more than the " + std::to_string(kScratchBytes) +
                        "-byte static scratch; use wn_conv3d_wgrad with a workspace")
                           .c_str());
    void* ws = nullptr;
    if (int rc = scratch_for_current_device(&ws)) return rc;
    const WgradPlan pl = wgrad_plan(n, d, h, w, ci, co, k);
    launch_wgrad(pl, x, ci, dy, co, Grid3{n, d, h, w}, k, (float*)ws, (hipStream_t)stream);
    const long long nw = (long long)co * k * k * k * ci;
    hipLaunchKernelGGL(sum_chunks, dim3((unsigned)((nw + 15) / 16)), dim3(256), 0, (hipStream_t)stream,
                       (const float*)ws, pl.nchunk, nw, dW);
    return hip_result("conv_wgrad_noalloc");
}

size_t wn_bias_grad_workspace_bytes(long long V, int co) {
    if (V < 1 || co < 1 || co > 256) return 0;
    return (size_t)((V + bg_rows(co) - 1) / bg_rows(co)) * (size_t)co * sizeof(float);
}

int wn_bias_grad(const float* dy, long long V, int co, float* db, void* workspace, size_t workspace_bytes,
                 void* stream) {
    if (!dy || !db || V < 1 || co < 1 || co > 256) return err(-1, "wn_bias_grad: bad arguments");
    if (!workspace || workspace_bytes < wn_bias_grad_workspace_bytes(V, co))
        return err(-1, "wn_bias_grad: workspace too small");
    const long long nblk = (V + bg_rows(co) - 1) / bg_rows(co);
    if (nblk > (1LL << 31) - 1) return err(-1, "wn_bias_grad: too many voxels");
    hipLaunchKernelGGL(bias_grad_part, dim3((unsigned)nblk), dim3(256), 0, (hipStream_t)stream, dy, V, co,
                       (float*)workspace);
    hipLaunchKernelGGL(bias_grad_final, dim3(co), dim3(256), 0, (hipStream_t)stream, (const float*)workspace,
                       (int)nblk, co, db);
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
