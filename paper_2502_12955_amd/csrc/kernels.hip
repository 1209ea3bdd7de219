// HIP kernels of the multi-component Shan-Chen LBM with reactive solute (gfx950).
//
// State: pre-collision populations in buffer A, structure of arrays
// f[s][i][n] and h[k][n], node n = x + nx*(y + ny*z).  One step reads A and
// writes B with push streaming (reads of a node's own populations are
// coalesced; writes go to n + c_i, or back to n for a solid downstream node:
// halfway bounce-back).  The caller swaps A and B after each step.
//
// Per fluid node (paper, multi-component LBM section):
//   rho_s = sum_i f^s_i (eq:1.7); psi_s = rho0 (1 - exp(-rho_s/rho0)) (eq:1.11)
//   F^s = -psi_s sum_t G_st sum_i w_i psi_t(x+c_i) c_i          (eq:1.14)
//         -G_ads,s rho_s sum_i w_i s(x+c_i) c_i                  (eq:1.15)
//         +rho_s accel
//   u = (sum_s j_s + F^s/2) / rho                                (eq:1.19)
//   Guo: u^eq_s = u, source eq:1.21 times (1 - 1/(2 tau_s))      (eq:1.16)
//   SC:  u^eq_s = u' + tau_s F^s/rho_s, u' of eq:1.18, no source (eq:1.17)
//   f*_i = f_i + (f^eq_i(rho_s, u^eq_s) - f_i)/tau_s [+ source]   (eq:6, eq:1.16)
// Solute: C = sum_k h_k, h*_k = h_k + (W_k C (1 + e_k.u/cs2) - h_k)/tau_d
// (eq:therpop_species); wet links get h_k = 2 W C_b - h_in with
// C_b = 2 h_in/(2W + k tau_d/(tau_d - 1/2)) (eq:wetnode9, per missing link);
// inlet x = 0: h_+x = 2 W C_in - h_-x; outlet x = nx-1: h_-x keeps its own
// post-collision value (zero gradient).

#include <math.h>

#include "common.hpp"
#include "kernels.hpp"
#include "node.hpp"

namespace mclbm {

// ---------------------------------------------------------------------------
// two-pass variant: (1) pseudo-potential field, (2) collide + push
// ---------------------------------------------------------------------------
template <int LAT, int ST, int NC>
__global__ void __launch_bounds__(256) k_density_psi(Phys<typename Store<ST>::R> P, long long N,
                                                     const typename Store<ST>::T* __restrict__ fA,
                                                     const uint32_t* __restrict__ links,
                                                     typename Store<ST>::R* __restrict__ psi) {
    using L = Lat<LAT>;
    using S = Store<ST>;
    using R = typename S::R;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= P.nx) return;
    const long long n = x + (long long)P.nx * (blockIdx.y + (long long)P.ny * blockIdx.z);
    const uint32_t lw = links[n];
    R sh[NC][L::Q];
    load_shifts<LAT, ST, NC>(P, sh);
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        R out = 0;
        if (!(lw & SOLID_BIT)) {
            R r = 0;
#pragma unroll
            for (int i = 0; i < L::Q; ++i) r += S::load(plane(fA, N, s * L::Q + i) + n, sh[s][i]);
            out = P.rho0 * (R(1) - exp_r<R>(-r * P.inv_rho0));
        }
        plane(psi, N, s)[n] = out;
    }
}

template <int LAT, int ST, int NC>
__global__ void __launch_bounds__(256) k_collide_push(Phys<typename Store<ST>::R> P, long long N,
                                                      const typename Store<ST>::T* __restrict__ fA,
                                                      typename Store<ST>::T* __restrict__ fB,
                                                      const typename Store<ST>::T* __restrict__ hA,
                                                      typename Store<ST>::T* __restrict__ hB,
                                                      const uint32_t* __restrict__ links,
                                                      const typename Store<ST>::R* __restrict__ psi) {
    using L = Lat<LAT>;
    using S = Store<ST>;
    using R = typename S::R;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= P.nx) return;
    const int y = blockIdx.y, z = blockIdx.z;
    const long long n = x + (long long)P.nx * (y + (long long)P.ny * z);
    const uint32_t lw = links[n];
    if (lw & SOLID_BIT) return;
    R sh[NC][L::Q];
    load_shifts<LAT, ST, NC>(P, sh);
    R f[NC][L::Q];
#pragma unroll
    for (int s = 0; s < NC; ++s)
#pragma unroll
        for (int i = 0; i < L::Q; ++i) f[s][i] = S::load(plane(fA, N, s * L::Q + i) + n, sh[s][i]);
    R u[3];
    auto nb = [&](int t, int i) -> R { return plane(psi, N, t)[nb_index<LAT>(P, x, y, z, i)]; };
    flow_collide<LAT, NC, R>(P, lw, f, nb, u);
    flow_push<LAT, ST, NC>(P, lw, x, y, z, n, N, fB, f, sh);
    if (P.solute) {
        R h[L::QS];
#pragma unroll
        for (int k = 0; k < L::QS; ++k) h[k] = S::load_plain(plane(hA, N, k) + n);
        solute_collide<LAT, R>(P, h, u);
        solute_push<LAT, ST>(P, lw, x, y, z, n, N, hB, h);
    }
}

// ---------------------------------------------------------------------------
// initialisation at equilibrium (no force term); solid slots get 0
// ---------------------------------------------------------------------------
template <int LAT, int ST, int NC>
__global__ void __launch_bounds__(256) k_init_eq(Phys<typename Store<ST>::R> P, long long N,
                                                 typename Store<ST>::T* __restrict__ fA,
                                                 typename Store<ST>::T* __restrict__ hA,
                                                 const uint32_t* __restrict__ links,
                                                 const double* __restrict__ rho, const double* __restrict__ u,
                                                 const double* __restrict__ C) {
    using L = Lat<LAT>;
    using S = Store<ST>;
    using R = typename S::R;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= P.nx) return;
    const long long n = x + (long long)P.nx * (blockIdx.y + (long long)P.ny * blockIdx.z);
    const bool solid = links[n] & SOLID_BIT;
    R sh[NC][L::Q];
    load_shifts<LAT, ST, NC>(P, sh);
    R v[3] = {0, 0, 0};
    if (u && !solid) {
        v[0] = (R)u[n];
        v[1] = (R)u[N + n];
        v[2] = (R)u[2 * N + n];
    }
    const R vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        const R r = solid ? R(0) : (R)rho[s * N + n];
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            const R cv = R(L::cx[i]) * v[0] + R(L::cy[i]) * v[1] + R(L::cz[i]) * v[2];
            const R feq = wgt<LAT, R>(i) * r * (R(1) + R(3) * cv + R(4.5) * cv * cv - R(1.5) * vv);
            if (solid) S::store_plain(plane(fA, N, s * L::Q + i) + n, R(0));
            else S::store(plane(fA, N, s * L::Q + i) + n, feq, sh[s][i]);
        }
    }
    if (P.solute) {
        const R c0 = (C && !solid) ? (R)C[n] : R(0);
#pragma unroll
        for (int k = 0; k < L::QS; ++k) {
            const R W = (k == 0) ? P.Ws0 : P.Ws;
            const R eu = R(L::cx[k]) * v[0] + R(L::cy[k]) * v[1] + R(L::cz[k]) * v[2];
            S::store_plain(plane(hA, N, k) + n, solid ? R(0) : W * c0 * (R(1) + eu * P.inv_cs2s));
        }
    }
}

// ---------------------------------------------------------------------------
// moments of the current state: rho_s, barycentric u with half force, C.
// Reuses flow_collide for the force and velocity (the post-collision values
// it leaves in the local copy are discarded).
// ---------------------------------------------------------------------------
template <int LAT, int ST, int NC>
__device__ __forceinline__ void node_moments(const Phys<typename Store<ST>::R>& P, long long N, int x, int y,
                                             int z, long long n, uint32_t lw,
                                             const typename Store<ST>::T* __restrict__ fA,
                                             const typename Store<ST>::T* __restrict__ hA,
                                             const typename Store<ST>::R* __restrict__ psi,
                                             typename Store<ST>::R (&rho)[NC], typename Store<ST>::R (&u)[3],
                                             typename Store<ST>::R& C) {
    using L = Lat<LAT>;
    using S = Store<ST>;
    using R = typename S::R;
    R sh[NC][L::Q];
    load_shifts<LAT, ST, NC>(P, sh);
    R f[NC][L::Q];
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        R r = 0;
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            f[s][i] = S::load(plane(fA, N, s * L::Q + i) + n, sh[s][i]);
            r += f[s][i];
        }
        rho[s] = r;
    }
    auto nb = [&](int t, int i) -> R { return plane(psi, N, t)[nb_index<LAT>(P, x, y, z, i)]; };
    flow_collide<LAT, NC, R>(P, lw, f, nb, u);
    C = 0;
    if (P.solute) {
#pragma unroll
        for (int k = 0; k < L::QS; ++k) C += S::load_plain(plane(hA, N, k) + n);
    }
}

template <int LAT, int ST, int NC>
__global__ void __launch_bounds__(256) k_moments_out(Phys<typename Store<ST>::R> P, long long N,
                                                     const typename Store<ST>::T* __restrict__ fA,
                                                     const typename Store<ST>::T* __restrict__ hA,
                                                     const uint32_t* __restrict__ links,
                                                     const typename Store<ST>::R* __restrict__ psi,
                                                     double* __restrict__ rho_out, double* __restrict__ u_out,
                                                     double* __restrict__ C_out) {
    using R = typename Store<ST>::R;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= P.nx) return;
    const int y = blockIdx.y, z = blockIdx.z;
    const long long n = x + (long long)P.nx * (y + (long long)P.ny * z);
    const uint32_t lw = links[n];
    R rho[NC] = {}, u[3] = {0, 0, 0}, C = 0;
    if (!(lw & SOLID_BIT)) node_moments<LAT, ST, NC>(P, N, x, y, z, n, lw, fA, hA, psi, rho, u, C);
    if (rho_out)
        for (int s = 0; s < NC; ++s) rho_out[s * N + n] = (double)rho[s];
    if (u_out)
        for (int a = 0; a < 3; ++a) u_out[a * N + n] = (double)u[a];
    if (C_out) C_out[n] = (double)C;
}

// ---------------------------------------------------------------------------
// monitors: FP64 block partials, fixed-order reduction
//   v[0] mass_0  v[1] mass_1  v[2] mass_C  v[3] |du|^2  v[4] |u|^2
//   v[5] dphi^2  v[6] phi^2   v[7] dC^2    v[8] C^2     v[9] non-finite
//   v[10] fluid nodes
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int LAT, int ST, int NC>
__global__ void __launch_bounds__(256) k_monitor(Phys<typename Store<ST>::R> P, long long N,
                                                 const typename Store<ST>::T* __restrict__ fA,
                                                 const typename Store<ST>::T* __restrict__ hA,
                                                 const uint32_t* __restrict__ links,
                                                 const typename Store<ST>::R* __restrict__ psi,
                                                 typename Store<ST>::R* __restrict__ snap, int have_snapshot,
                                                 double* __restrict__ partials) {
    using R = typename Store<ST>::R;
    __shared__ double red[MON_NV][4];
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y, z = blockIdx.z;
    double v[MON_NV];
#pragma unroll
    for (int k = 0; k < MON_NV; ++k) v[k] = 0.0;
    if (x < P.nx) {
        const long long n = x + (long long)P.nx * (y + (long long)P.ny * z);
        const uint32_t lw = links[n];
        if (!(lw & SOLID_BIT)) {
            R rho[NC], u[3], C;
            node_moments<LAT, ST, NC>(P, N, x, y, z, n, lw, fA, hA, psi, rho, u, C);
            R phi = 0;
            if (NC == 2) {
                const R tot = rho[0] + rho[NC - 1];
                phi = (tot != R(0)) ? (rho[0] - rho[NC - 1]) / tot : R(0);
            }
            v[0] = rho[0];
            v[1] = (NC == 2) ? (double)rho[NC - 1] : 0.0;
            v[2] = C;
            double uu = 0, du = 0;
            for (int a = 0; a < 3; ++a) {
                const double ua = u[a];
                uu += ua * ua;
                if (have_snapshot) {
                    const double d = ua - (double)plane(snap, N, a)[n];
                    du += d * d;
                }
                plane(snap, N, a)[n] = u[a];
            }
            v[3] = du;
            v[4] = uu;
            if (have_snapshot) {
                const double dp = (double)phi - (double)plane(snap, N, 3)[n];
                const double dc = (double)C - (double)plane(snap, N, 4)[n];
                v[5] = dp * dp;
                v[7] = dc * dc;
            }
            v[6] = (double)phi * (double)phi;
            v[8] = (double)C * (double)C;
            plane(snap, N, 3)[n] = phi;
            plane(snap, N, 4)[n] = C;
            bool bad = !isfinite((double)rho[0]) || !isfinite((double)rho[NC - 1]) || !isfinite((double)C) ||
                       !isfinite((double)u[0]) || !isfinite((double)u[1]) || !isfinite((double)u[2]);
            v[9] = bad ? 1.0 : 0.0;
            v[10] = 1.0;
        }
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < MON_NV; ++k) {
        const double s = wave_sum(v[k]);
        if (lane == 0) red[k][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x < MON_NV) {
        const int nw = (blockDim.x + 63) >> 6;
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[threadIdx.x][w];
        const long long b = blockIdx.x + (long long)gridDim.x * (blockIdx.y + (long long)gridDim.y * blockIdx.z);
        partials[b * MON_NV + threadIdx.x] = s;
    }
}

// one block of 256 threads: thread t sums rows b = t, t+256, ... in order,
// then a fixed tree over the 256 threads
__global__ void __launch_bounds__(256) k_monitor_final(const double* __restrict__ partials, long long nblocks,
                                                       double* __restrict__ result) {
    __shared__ double acc[256][MON_NV + 1];
    const int t = threadIdx.x;
    double s[MON_NV];
#pragma unroll
    for (int k = 0; k < MON_NV; ++k) s[k] = 0.0;
    for (long long b = t; b < nblocks; b += 256)
#pragma unroll
        for (int k = 0; k < MON_NV; ++k) s[k] += partials[b * MON_NV + k];
#pragma unroll
    for (int k = 0; k < MON_NV; ++k) acc[t][k] = s[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
#pragma unroll
            for (int k = 0; k < MON_NV; ++k) acc[t][k] += acc[t + w][k];
        __syncthreads();
    }
    if (t < MON_NV) result[t] = acc[0][t];
}

// ---------------------------------------------------------------------------
// host dispatch
// ---------------------------------------------------------------------------
template <typename R>
Phys<R> make_phys(const Ctx& c) {
    Phys<R> P;
    P.nx = c.nx;
    P.ny = c.ny;
    P.nz = c.nz;
    P.forcing = c.forcing;
    P.solute = c.solute;
    for (int s = 0; s < 2; ++s) {
        const double tau = c.tau[s] > 0 ? c.tau[s] : 1.0;
        P.tau[s] = (R)tau;
        P.inv_tau[s] = (R)(1.0 / tau);
        P.lam[s] = (R)(1.0 - 1.0 / (2.0 * tau));
        for (int t = 0; t < 2; ++t) P.G[s][t] = (R)c.G[s][t];
        P.Gads[s] = (R)c.Gads[s];
        for (int i = 0; i < 19; ++i) P.sh[s][i] = (R)shift_f32(c, s, i);
    }
    P.rho0 = (R)c.rho0;
    P.inv_rho0 = (R)(1.0 / c.rho0);
    for (int a = 0; a < 3; ++a) P.accel[a] = (R)c.accel[a];
    const int QS = (c.lat == 1) ? 7 : 5;
    const double Ws = (1.0 - c.J0) / (double)(QS - 1);
    const double cs2s = 2.0 * Ws;
    const double tau_d = (c.D > 0 ? c.D : 1.0) / cs2s + 0.5;
    P.Ws0 = (R)c.J0;
    P.Ws = (R)Ws;
    P.inv_cs2s = (R)(1.0 / cs2s);
    P.inv_tau_d = (R)(1.0 / tau_d);
    P.wet_inv_den = (R)(1.0 / (2.0 * Ws + c.k_wall * tau_d / (tau_d - 0.5)));
    P.C_in = (R)c.C_in;
    return P;
}

template Phys<float> make_phys<float>(const Ctx&);
template Phys<double> make_phys<double>(const Ctx&);

template <int ST>
using SR = typename Store<ST>::R;
template <int ST>
using STT = typename Store<ST>::T;

static inline dim3 node_block(const Ctx& c) { return dim3(c.nx >= 256 ? 256 : (c.nx >= 128 ? 128 : 64)); }
static inline dim3 node_grid(const Ctx& c) {
    const dim3 b = node_block(c);
    return dim3((c.nx + b.x - 1) / b.x, c.ny, c.nz);
}

size_t monitor_blocks(const Ctx& c) {
    const dim3 g = node_grid(c);
    return (size_t)g.x * g.y * g.z;
}

float shift_f32(const Ctx& c, int s, int i) {
    if (c.st < ST_F16S) return 0.0f;
    static const int wn19[19] = {12, 2, 2, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
    static const int wn9[9] = {16, 4, 4, 4, 4, 1, 1, 1, 1};
    const int wn = (c.lat == 1) ? wn19[i] : wn9[i];
    if (i >= ((c.lat == 1) ? 19 : 9)) return 0.0f;
    const float w = (float)wn / 36.0f;
    return w * (float)c.rhobar[s];
}

template <int LAT, int ST, int NC>
static hipError_t step_two_pass(const Ctx& c) {
    auto P = make_phys<SR<ST>>(c);
    const dim3 b = node_block(c), g = node_grid(c);
    hipLaunchKernelGGL((k_density_psi<LAT, ST, NC>), g, b, 0, c.stream, P, c.N, (const STT<ST>*)c.fA, c.links,
                       (SR<ST>*)c.psi);
    hipLaunchKernelGGL((k_collide_push<LAT, ST, NC>), g, b, 0, c.stream, P, c.N, (const STT<ST>*)c.fA,
                       (STT<ST>*)c.fB, (const STT<ST>*)c.hA, (STT<ST>*)c.hB, c.links, (const SR<ST>*)c.psi);
    return hipGetLastError();
}

template <int LAT, int ST, int NC>
static hipError_t init_t(const Ctx& c, const double* rho, const double* u, const double* C) {
    auto P = make_phys<SR<ST>>(c);
    hipLaunchKernelGGL((k_init_eq<LAT, ST, NC>), node_grid(c), node_block(c), 0, c.stream, P, c.N,
                       (STT<ST>*)c.fA, (STT<ST>*)c.hA, c.links, rho, u, C);
    return hipGetLastError();
}

template <int LAT, int ST, int NC>
static hipError_t moments_t(const Ctx& c, double* rho, double* u, double* C) {
    auto P = make_phys<SR<ST>>(c);
    const dim3 b = node_block(c), g = node_grid(c);
    hipLaunchKernelGGL((k_density_psi<LAT, ST, NC>), g, b, 0, c.stream, P, c.N, (const STT<ST>*)c.fA, c.links,
                       (SR<ST>*)c.psi);
    hipLaunchKernelGGL((k_moments_out<LAT, ST, NC>), g, b, 0, c.stream, P, c.N, (const STT<ST>*)c.fA,
                       (const STT<ST>*)c.hA, c.links, (const SR<ST>*)c.psi, rho, u, C);
    return hipGetLastError();
}

template <int LAT, int ST, int NC>
static hipError_t monitor_t(const Ctx& c, int have_snapshot) {
    auto P = make_phys<SR<ST>>(c);
    const dim3 b = node_block(c), g = node_grid(c);
    hipLaunchKernelGGL((k_density_psi<LAT, ST, NC>), g, b, 0, c.stream, P, c.N, (const STT<ST>*)c.fA, c.links,
                       (SR<ST>*)c.psi);
    hipLaunchKernelGGL((k_monitor<LAT, ST, NC>), g, b, 0, c.stream, P, c.N, (const STT<ST>*)c.fA,
                       (const STT<ST>*)c.hA, c.links, (const SR<ST>*)c.psi, (SR<ST>*)c.snap, have_snapshot,
                       c.partials);
    hipLaunchKernelGGL(k_monitor_final, dim3(1), dim3(256), 0, c.stream, (const double*)c.partials,
                       (long long)monitor_blocks(c), c.result);
    return hipGetLastError();
}

// fused kernel (defined in fused.hip)
template <int LAT, int ST, int NC>
hipError_t step_fused(const Ctx& c);

#define MCLBM_DISPATCH(FN, ...)                                                             \
    do {                                                                                    \
        const int key = c.lat * 100 + c.st * 10 + c.nc;                                     \
        switch (key) {                                                                      \
            case 1: return FN<0, 0, 1>(__VA_ARGS__);                                        \
            case 2: return FN<0, 0, 2>(__VA_ARGS__);                                        \
            case 11: return FN<0, 1, 1>(__VA_ARGS__);                                       \
            case 12: return FN<0, 1, 2>(__VA_ARGS__);                                       \
            case 21: return FN<0, 2, 1>(__VA_ARGS__);                                       \
            case 22: return FN<0, 2, 2>(__VA_ARGS__);                                       \
            case 31: return FN<0, 3, 1>(__VA_ARGS__);                                       \
            case 32: return FN<0, 3, 2>(__VA_ARGS__);                                       \
            case 101: return FN<1, 0, 1>(__VA_ARGS__);                                      \
            case 102: return FN<1, 0, 2>(__VA_ARGS__);                                      \
            case 111: return FN<1, 1, 1>(__VA_ARGS__);                                      \
            case 112: return FN<1, 1, 2>(__VA_ARGS__);                                      \
            case 121: return FN<1, 2, 1>(__VA_ARGS__);                                      \
            case 122: return FN<1, 2, 2>(__VA_ARGS__);                                      \
            case 131: return FN<1, 3, 1>(__VA_ARGS__);                                      \
            case 132: return FN<1, 3, 2>(__VA_ARGS__);                                      \
            default: return hipErrorInvalidValue;                                           \
        }                                                                                   \
    } while (0)

hipError_t k_init(const Ctx& c, const double* rho, const double* u, const double* C) {
    MCLBM_DISPATCH(init_t, c, rho, u, C);
}

hipError_t k_step(const Ctx& c) {
    if (c.variant == 1) MCLBM_DISPATCH(step_two_pass, c);
    MCLBM_DISPATCH(step_fused, c);
}

hipError_t k_moments(const Ctx& c, double* rho, double* u, double* C) { MCLBM_DISPATCH(moments_t, c, rho, u, C); }

hipError_t k_monitor(const Ctx& c, int have_snapshot) { MCLBM_DISPATCH(monitor_t, c, have_snapshot); }

}  // namespace mclbm
