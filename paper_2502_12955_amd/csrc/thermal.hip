// Conjugate heat transfer kernels (paper, Reactive LBM subsection): the solid
// energy pass and the interface solve that follow the collide pass of a step,
// plus initialisation and output.  The fluid energy populations are collided
// and pushed by the collide pass itself (with the flow).
//
// Node lists (single lattice): the fluid list of the flow; the solid list =
// solid nodes and interface nodes (fluid nodes with a solid flow-lattice
// neighbour), numbered like the fluid list, with smap (box -> solid-list
// index, -1 for a fluid node without solid populations); the interface list
// of (fluid index, solid-list index, bits of the solid populations whose
// upstream node has no solid populations).
//
// Per step, after the collide pass has written buffer B:
//   k_th_solid:  gs_i <- gs_i - (gs_i - w_i E_s) / tau_es (eq:therpop_solid,
//                eq:therpopeq_solid), pushed to neighbours that carry solid
//                populations (a population heading into pure fluid leaves).
//   k_th_iface:  at every interface node, the unknowns g_i = w_i X_f (upstream
//                solid) and gs_i = w_i X_s (upstream pure fluid) from
//                  (Kn_f + W_f X_f) / rc_f = (Kn_s + W_s X_s) / rc_s
//                  k_f (W_f' X_f - B_f) = k_s (A_s - W_s' X_s) + Hdot
//                (eq:countSlipTempCon, eq:countSlipFluxCon; W' and B / A over
//                the unknowns whose opposite is known), Hdot = h_r sum over the
//                node's wet solute links of k(T) C_b (eq:reacRate) with
//                C_b = 2 h_in / (2 W + k(T) tau_d / (tau_d - 1/2)) (eq:wetnode9),
//                k(T) = A exp(-E/R / T), iterated on T = (Kn_f + W_f X_f) / rc_f
//                until it settles; then the solute's wet-link populations
//                (and the product's) with the rate of the last iteration.
// For a flat wall this is exactly eq:unknownpopTempS and eq:unknownpopTempF.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "common.hpp"
#include "kernels.hpp"
#include "node.hpp"

namespace mclbm {
namespace {

template <typename R>
struct ThP {
    int nx, ny, nz;
    int solute, product;
    int nsolid, niface, nfluid;
    int maxit;
    R inv_tau_es, kf, ks, cfs, rc_f, rc_s, h_r, A, EoR, tol;
    R Ws;          // solute link weight
    R wet_fac;     // tau_d / (tau_d - 1/2)
    R prod_fac;    // tau_d2 / (tau_d2 - 1/2)
};

template <int LAT, int ST>
__global__ void __launch_bounds__(256) k_th_solid(ThP<typename Store<ST>::R> P, const int* __restrict__ smap,
                                                  const unsigned* __restrict__ spos,
                                                  const typename Store<ST>::T* __restrict__ gsA,
                                                  typename Store<ST>::T* __restrict__ gsB) {
    using L = Lat<LAT>;
    using S = Store<ST>;
    using R = typename S::R;
    constexpr int Q = L::Q;
    const unsigned j = blockIdx.x * blockDim.x + threadIdx.x;
    if ((int)j >= P.nsolid) return;
    R g[Q];
    R E = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        g[i] = S::load_plain(blk(gsA, Q, i, j));
        E += g[i];
    }
    int x, y, z;
    coords(spos[j], P.nx, P.ny, x, y, z);
    const NbIdx nb = make_nb(x, y, z, P.nx, P.ny, P.nz);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const R post = g[i] - (g[i] - wgt<LAT, R>(i) * E) * P.inv_tau_es;
        if (i == 0) {
            S::store_plain(blk(gsB, Q, 0, j), post);
        } else {
            const int m = smap[nb.at(L::cx[i], L::cy[i], L::cz[i])];
            if (m >= 0) S::store_plain(blk(gsB, Q, i, (unsigned)m), post);
        }
    }
}

template <int LAT, int ST, int PR>
__global__ void __launch_bounds__(256) k_th_iface(ThP<typename Store<ST>::R> P, const int* __restrict__ iface,
                                                  const uint32_t* __restrict__ links,
                                                  typename Store<ST>::T* __restrict__ gB,
                                                  typename Store<ST>::T* __restrict__ gsB,
                                                  typename Store<ST>::T* __restrict__ hB, int hplanes,
                                                  typename Store<ST>::R* __restrict__ Ti,
                                                  unsigned long long* __restrict__ stats) {
    using L = Lat<LAT>;
    using S = Store<ST>;
    using R = typename S::R;
    constexpr int Q = L::Q, QS = L::QS;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= P.niface) return;
    const unsigned k = (unsigned)iface[4 * q], j = (unsigned)iface[4 * q + 1];
    const uint32_t msb = (uint32_t)iface[4 * q + 2];   // bit i: solid unknown
    const uint32_t lw = links[k];                        // bit i: fluid unknown (upstream solid)
    R g[Q], gs[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        g[i] = S::load_plain(blk(gB, Q, i, k));
        gs[i] = S::load_plain(blk(gsB, Q, i, j));
    }
    R Knf = 0, Kns = 0, Wf = 0, Ws = 0, Wfp = 0, Wsp = 0, Bf = 0, As = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int o = L::opp[i];
        const bool mf = i > 0 && (lw >> i) & 1u, mfo = o > 0 && (lw >> o) & 1u;
        const bool ms = i > 0 && (msb >> i) & 1u, mso = o > 0 && (msb >> o) & 1u;
        const R w = wgt<LAT, R>(i);
        if (mf) {
            Wf += w;
            if (!mfo) {
                Wfp += w;
                Bf += g[o];
            }
        } else {
            Knf += g[i];
        }
        if (ms) {
            Ws += w;
            if (!mso) {
                Wsp += w;
                As += gs[o];
            }
        } else {
            Kns += gs[i];
        }
    }
    const R det = Wf * P.ks * Wsp + P.cfs * Ws * P.kf * Wfp;
    const bool degenerate = !(det > R(0));
    // wet solute links of this node and their incoming populations
    R hin[QS], Cb[QS];
    uint32_t wet = 0;
    if (P.solute) {
#pragma unroll
        for (int d = 1; d < QS; ++d)
            if (lw & (1u << (L::WET_SHIFT + d))) {
                wet |= 1u << d;
                hin[d] = S::load_plain(blk(hB, hplanes, L::opp[d], k));
            }
    }
    R T = Ti[q], Xf = 0, Xs = 0, kr = 0;
    int it = 0;
    bool settled = false;
    while (it < P.maxit) {
        ++it;
        kr = P.A * exp_r<R>(-P.EoR / T);
        R Hdot = 0;
#pragma unroll
        for (int d = 1; d < QS; ++d)
            if (wet & (1u << d)) {
                Cb[d] = R(2) * hin[d] / (R(2) * P.Ws + kr * P.wet_fac);
                Hdot += P.h_r * kr * Cb[d];
            }
        if (!degenerate)
            Xs = (Wf * (P.ks * As + P.kf * Bf + Hdot) - P.kf * Wfp * (P.cfs * Kns - Knf)) / det;
        else
            Xs = Ws > R(0) ? Kns / (R(1) - Ws) : R(0);
        Xf = (P.cfs * (Kns + Ws * Xs) - Knf) / Wf;
        const R Tn = (Knf + Wf * Xf) / P.rc_f;
        const bool done = fabs(Tn - T) <= P.tol * fabs(Tn);
        T = Tn;
        if (done) {
            settled = true;
            break;
        }
    }
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        if ((lw >> i) & 1u) S::store_plain(blk(gB, Q, i, k), wgt<LAT, R>(i) * Xf);
        if ((msb >> i) & 1u) S::store_plain(blk(gsB, Q, i, j), wgt<LAT, R>(i) * Xs);
    }
    Ti[q] = T;
#pragma unroll
    for (int d = 1; d < QS; ++d)
        if (wet & (1u << d)) {
            S::store_plain(blk(hB, hplanes, d, k), R(2) * P.Ws * Cb[d] - hin[d]);
            if (PR) {
                const R hin2 = S::load_plain(blk(hB, hplanes, QS + L::opp[d], k));
                S::store_plain(blk(hB, hplanes, QS + d, k), hin2 + kr * P.prod_fac * Cb[d]);
            }
        }
    atomicAdd(stats, (unsigned long long)it);
    if (!settled) atomicAdd(stats + 1, 1ull);
}

// initial energy populations from FP64 box fields
template <int LAT, int ST>
__global__ void __launch_bounds__(256) k_th_init(ThP<typename Store<ST>::R> P, const unsigned* __restrict__ pos,
                                                 const unsigned* __restrict__ spos, const int* __restrict__ iface,
                                                 const double* __restrict__ T, const double* __restrict__ u,
                                                 long long N, typename Store<ST>::T* __restrict__ gA,
                                                 typename Store<ST>::T* __restrict__ gsA,
                                                 typename Store<ST>::R* __restrict__ Ti) {
    using L = Lat<LAT>;
    using S = Store<ST>;
    using R = typename S::R;
    constexpr int Q = L::Q;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < P.nfluid) {
        const unsigned n = pos[t];
        R v[3] = {0, 0, 0};
        if (u) {
            v[0] = (R)u[n];
            v[1] = (R)u[N + n];
            v[2] = (R)u[2 * N + n];
        }
        const R E = P.rc_f * (R)T[n];
        const R uu = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const R cu = cdot<LAT, R>(i, v[0], v[1], v[2]);
            S::store_plain(blk(gA, Q, i, (unsigned)t), wgt<LAT, R>(i) * E * (R(1) + R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu));
        }
    }
    if (t < P.nsolid) {
        const R Es = P.rc_s * (R)T[spos[t]];
#pragma unroll
        for (int i = 0; i < Q; ++i) S::store_plain(blk(gsA, Q, i, (unsigned)t), wgt<LAT, R>(i) * Es);
    }
    if (t < P.niface) Ti[t] = (R)T[pos[iface[4 * t]]];
}

// what 0: temperature of every node; 1: fluid energy plane `plane` at fluid
// nodes; 2: solid energy plane at solid-list nodes (dst pre-filled with 0)
template <int LAT, int ST>
__global__ void __launch_bounds__(256) k_th_out(ThP<typename Store<ST>::R> P, const unsigned* __restrict__ pos,
                                                const unsigned* __restrict__ spos, const int* __restrict__ map,
                                                const typename Store<ST>::T* __restrict__ gA,
                                                const typename Store<ST>::T* __restrict__ gsA, int what, int plane,
                                                double* __restrict__ dst) {
    using L = Lat<LAT>;
    using S = Store<ST>;
    using R = typename S::R;
    constexpr int Q = L::Q;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (what == 0) {
        if (t < P.nfluid) {
            R E = 0;
            for (int i = 0; i < Q; ++i) E += S::load_plain(blk(gA, Q, i, (unsigned)t));
            dst[pos[t]] = (double)(E / P.rc_f);
        }
        if (t < P.nsolid && map[spos[t]] < 0) {   // solid node (interface nodes report the fluid side)
            R E = 0;
            for (int i = 0; i < Q; ++i) E += S::load_plain(blk(gsA, Q, i, (unsigned)t));
            dst[spos[t]] = (double)(E / P.rc_s);
        }
    } else if (what == 1) {
        if (t < P.nfluid) dst[pos[t]] = (double)S::load_plain(blk(gA, Q, plane, (unsigned)t));
    } else {
        if (t < P.nsolid) dst[spos[t]] = (double)S::load_plain(blk(gsA, Q, plane, (unsigned)t));
    }
}

template <typename R>
ThP<R> make_thp(const Ctx& c, int Q, int QS) {
    ThP<R> P;
    P.nx = c.thermal_nx;
    P.ny = c.thermal_ny;
    P.nz = c.thermal_nz;
    P.solute = c.solute;
    P.product = c.product;
    P.nsolid = (int)c.nsolid;
    P.niface = (int)c.niface;
    P.nfluid = (int)c.thermal_nfluid;
    P.maxit = c.th_maxit;
    P.inv_tau_es = (R)(1.0 / c.th_tau_es);
    P.kf = (R)(1.0 - 0.5 / c.th_tau_ef);
    P.ks = (R)(1.0 - 0.5 / c.th_tau_es);
    P.cfs = (R)(c.th_rhocp_f / c.th_rhocp_s);
    P.rc_f = (R)c.th_rhocp_f;
    P.rc_s = (R)c.th_rhocp_s;
    P.h_r = (R)c.th_h_r;
    P.A = (R)c.th_A;
    P.EoR = (R)c.th_EoR;
    const double eps = sizeof(R) == 8 ? 2.220446049250313e-16 : 1.1920928955078125e-07;
    P.tol = (R)(c.th_tol > 4.0 * eps ? c.th_tol : 4.0 * eps);
    const double Ws = (1.0 - c.J0) / (double)(QS - 1), cs2s = 2.0 * Ws;
    const double tau_d = (c.D > 0 ? c.D : 1.0) / cs2s + 0.5;
    const double tau_d2 = (c.D2 > 0 ? c.D2 : 1.0) / cs2s + 0.5;
    P.Ws = (R)Ws;
    P.wet_fac = (R)(tau_d / (tau_d - 0.5));
    P.prod_fac = (R)(tau_d2 / (tau_d2 - 0.5));
    (void)Q;
    return P;
}

inline dim3 blocks(long long n) { return dim3((unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1)); }

template <int LAT, int ST>
hipError_t step_th(const Ctx& c) {
    using S = Store<ST>;
    using R = typename S::R;
    using T = typename S::T;
    const ThP<R> P = make_thp<R>(c, Lat<LAT>::Q, Lat<LAT>::QS);
    if (P.nsolid > 0)
        hipLaunchKernelGGL((k_th_solid<LAT, ST>), blocks(P.nsolid), dim3(256), 0, c.stream, P, c.smap, c.spos,
                           (const T*)c.gsA, (T*)c.gsB);
    if (P.niface > 0) {
        if (c.product)
            hipLaunchKernelGGL((k_th_iface<LAT, ST, 1>), blocks(P.niface), dim3(256), 0, c.stream, P, c.iface, c.links,
                               (T*)c.gB, (T*)c.gsB, (T*)c.hB, c.hplanes, (R*)c.Ti, c.th_stats);
        else
            hipLaunchKernelGGL((k_th_iface<LAT, ST, 0>), blocks(P.niface), dim3(256), 0, c.stream, P, c.iface, c.links,
                               (T*)c.gB, (T*)c.gsB, (T*)c.hB, c.hplanes, (R*)c.Ti, c.th_stats);
    }
    return hipGetLastError();
}

template <int LAT, int ST>
hipError_t init_th(const Ctx& c, const double* Tf, const double* u) {
    using S = Store<ST>;
    using R = typename S::R;
    using T = typename S::T;
    const ThP<R> P = make_thp<R>(c, Lat<LAT>::Q, Lat<LAT>::QS);
    const long long n = std::max((long long)P.nfluid, std::max((long long)P.nsolid, (long long)P.niface));
    hipLaunchKernelGGL((k_th_init<LAT, ST>), blocks(n), dim3(256), 0, c.stream, P, c.pos, c.spos, c.iface, Tf, u,
                       c.Ntot, (T*)c.gA, (T*)c.gsA, (R*)c.Ti);
    return hipGetLastError();
}

template <int LAT, int ST>
hipError_t out_th(const Ctx& c, int what, int plane, double* dst) {
    using S = Store<ST>;
    using R = typename S::R;
    using T = typename S::T;
    const ThP<R> P = make_thp<R>(c, Lat<LAT>::Q, Lat<LAT>::QS);
    const long long n = std::max((long long)P.nfluid, (long long)P.nsolid);
    hipLaunchKernelGGL((k_th_out<LAT, ST>), blocks(n), dim3(256), 0, c.stream, P, c.pos, c.spos, c.map,
                       (const T*)c.gA, (const T*)c.gsA, what, plane, dst);
    return hipGetLastError();
}

#define MCLBM_TH_DISPATCH(FN, ...)                         \
    do {                                                   \
        switch (c.lat * 10 + c.st) {                       \
            case 0: return FN<0, ST_F64>(__VA_ARGS__);     \
            case 1: return FN<0, ST_F32>(__VA_ARGS__);     \
            case 10: return FN<1, ST_F64>(__VA_ARGS__);    \
            case 11: return FN<1, ST_F32>(__VA_ARGS__);    \
            default: return hipErrorInvalidValue;          \
        }                                                  \
    } while (0)

}  // namespace

hipError_t k_thermal_step(const Ctx& c) { MCLBM_TH_DISPATCH(step_th, c); }
hipError_t k_thermal_init(const Ctx& c, const double* T, const double* u) { MCLBM_TH_DISPATCH(init_th, c, T, u); }
hipError_t k_thermal_out(const Ctx& c, int what, int plane, double* dst) {
    MCLBM_TH_DISPATCH(out_th, c, what, plane, dst);
}

}  // namespace mclbm
