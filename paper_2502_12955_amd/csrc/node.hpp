// Per-node device arithmetic shared by the flow kernels: the flow collision
// with interaction forces, the solute collision and the storage shifts.  See
// kernels.hip for the equations.
#pragma once

#include <math.h>

#include "common.hpp"

namespace mclbm {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ R exp_r(R v);
template <>
__device__ __forceinline__ double exp_r<double>(double v) { return exp(v); }
template <>
__device__ __forceinline__ float exp_r<float>(float v) { return expf(v); }

template <int LAT, typename R>
__device__ __forceinline__ R wgt(int i) { return R(Lat<LAT>::wn[i]) / R(36); }

// ---------------------------------------------------------------------------
// per-node flow collision (shared by all flow kernels)
//   f: pre-collision populations of the node (overwritten with post-collision)
//   psi_nb(t, i): pseudo-potential of component t at x + c_i; it must be 0
//                 for a solid neighbour (walls act through adhesion only)
//   lw: link word; u: barycentric velocity with half force (out)
// Arithmetic is arranged for few instructions: c_i has entries in {0, +-1},
// so every c.v is a compile-time selection of adds; the equilibrium is
// w rho (K + cv (3 + 4.5 cv)) with K = 1 - 1.5 v.v, and the Guo term is
// 3 w (cF (1 + 3 cu) - u.F).
// ---------------------------------------------------------------------------
template <int LAT>
struct LatMasks {
    // bits j (upstream-solid bits of the link word) grouped by c_ja sign and weight class
    static constexpr uint32_t mask(int a, int sign, int wn) {
        uint32_t m = 0;
        for (int j = 1; j < Lat<LAT>::Q; ++j) {
            const int c = a == 0 ? Lat<LAT>::cx[j] : (a == 1 ? Lat<LAT>::cy[j] : Lat<LAT>::cz[j]);
            if (c == sign && Lat<LAT>::wn[j] == wn) m |= 1u << j;
        }
        return m;
    }
};

template <int LAT>
__device__ __forceinline__ int ads36(uint32_t lw, int a) {
    // 36 * sum_i w_i s(x + c_i) c_ia = -sum_j wn_j c_ja bit_j   (bit j: x - c_j solid)
    constexpr int wa = (LAT == 1) ? 2 : 4;  // axis weight numerator
    using M = LatMasks<LAT>;
    const int pos = wa * __builtin_popcount(lw & M::mask(a, 1, wa)) + __builtin_popcount(lw & M::mask(a, 1, 1));
    const int neg = wa * __builtin_popcount(lw & M::mask(a, -1, wa)) + __builtin_popcount(lw & M::mask(a, -1, 1));
    return neg - pos;
}

template <int LAT, typename R>
__device__ __forceinline__ R cdot(int i, R x, R y, R z) {
    using L = Lat<LAT>;
    R r = R(0);
    if (L::cx[i] > 0) r = r + x;
    if (L::cx[i] < 0) r = r - x;
    if (L::cy[i] > 0) r = r + y;
    if (L::cy[i] < 0) r = r - y;
    if (LAT == 1) {
        if (L::cz[i] > 0) r = r + z;
        if (L::cz[i] < 0) r = r - z;
    }
    return r;
}

// FC: forcing scheme fixed at compile time (0 Guo, 1 Shan-Chen velocity
// shift) or -1 to follow P.forcing; the step kernel is compiled per scheme, so
// only one branch occupies its registers.
template <int LAT, int NC, typename R, class PsiNb, int FC = -1>
__device__ __forceinline__ void flow_collide(const Phys<R>& P, uint32_t lw, R (&f)[NC][Lat<LAT>::Q],
                                             PsiNb psi_nb, R (&u)[3]) {
    using L = Lat<LAT>;
    constexpr int Q = L::Q;
    R rho[NC], j[NC][3];
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        R r = 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) r += f[s][i];
        rho[s] = r;
        R jx = 0, jy = 0, jz = 0;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            if (L::cx[i] > 0) jx += f[s][i];
            if (L::cx[i] < 0) jx -= f[s][i];
            if (L::cy[i] > 0) jy += f[s][i];
            if (L::cy[i] < 0) jy -= f[s][i];
            if (L::cz[i] > 0) jz += f[s][i];
            if (L::cz[i] < 0) jz -= f[s][i];
        }
        j[s][0] = jx;
        j[s][1] = jy;
        j[s][2] = jz;
    }
    R psi_self[NC];
#pragma unroll
    for (int s = 0; s < NC; ++s) psi_self[s] = P.rho0 * (R(1) - exp_r<R>(-rho[s] * P.inv_rho0));

    // cohesion sums 36 * sum_i w_i psi_t(x + c_i) c_i
    R coh[NC][3];
#pragma unroll
    for (int t = 0; t < NC; ++t) {
        R cx = 0, cy = 0, cz = 0;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const R p = R(L::wn[i]) * psi_nb(t, i);
            if (L::cx[i] > 0) cx += p;
            if (L::cx[i] < 0) cx -= p;
            if (L::cy[i] > 0) cy += p;
            if (L::cy[i] < 0) cy -= p;
            if (L::cz[i] > 0) cz += p;
            if (L::cz[i] < 0) cz -= p;
        }
        coh[t][0] = cx;
        coh[t][1] = cy;
        coh[t][2] = cz;
    }
    R ads[3] = {0, 0, 0};
    if (P.Gads[0] != R(0) || (NC == 2 && P.Gads[NC - 1] != R(0))) {
#pragma unroll
        for (int a = 0; a < 3; ++a) ads[a] = R(ads36<LAT>(lw, a));
    }
    const R inv36 = R(1) / R(36);
    R F[NC][3];
#pragma unroll
    for (int s = 0; s < NC; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            R g = 0;
#pragma unroll
            for (int t = 0; t < NC; ++t) g += P.G[s][t] * coh[t][a];
            F[s][a] = (-psi_self[s] * g - P.Gads[s] * rho[s] * ads[a]) * inv36 + rho[s] * P.accel[a];
        }

    R rt = 0;
#pragma unroll
    for (int s = 0; s < NC; ++s) rt += rho[s];
    const R inv_rt = R(1) / rt;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        R m = 0;
#pragma unroll
        for (int s = 0; s < NC; ++s) m += j[s][a] + R(0.5) * F[s][a];
        u[a] = m * inv_rt;
    }

    // weights by class: rest, axis, diagonal (numerators of 36)
    constexpr int WN0 = L::wn[0], WN1 = L::wn[1], WN2 = L::wn[Q - 1];
    auto wclass = [](int i) { return i == 0 ? 0 : (L::wn[i] == WN1 ? 1 : 2); };
    const R w0 = R(WN0) / R(36), w1 = R(WN1) / R(36), w2 = R(WN2) / R(36);

    if (FC == 0 || (FC < 0 && P.forcing == 0)) {
        const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        const R K = R(1) - R(1.5) * uu;
        R wr[NC][3], lw3[NC][3], uF[NC], om[NC];
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            wr[s][0] = w0 * rho[s];
            wr[s][1] = w1 * rho[s];
            wr[s][2] = w2 * rho[s];
            const R l3 = R(3) * P.lam[s];
            lw3[s][0] = l3 * w0;
            lw3[s][1] = l3 * w1;
            lw3[s][2] = l3 * w2;
            uF[s] = u[0] * F[s][0] + u[1] * F[s][1] + u[2] * F[s][2];
            om[s] = P.inv_tau[s];
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int c = wclass(i);
            const R cu = cdot<LAT, R>(i, u[0], u[1], u[2]);
            const R t2 = cu * (R(4.5) * cu + R(3)) + K;
            const R t3 = R(3) * cu + R(1);
#pragma unroll
            for (int s = 0; s < NC; ++s) {
                const R cF = cdot<LAT, R>(i, F[s][0], F[s][1], F[s][2]);
                const R feq = wr[s][c] * t2;
                const R sp = cF * t3 - uF[s];
                f[s][i] = (f[s][i] + om[s] * (feq - f[s][i])) + lw3[s][c] * sp;
            }
        }
    } else {
        R num[3] = {0, 0, 0}, den = 0;
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            den += rho[s] * P.inv_tau[s];
#pragma unroll
            for (int a = 0; a < 3; ++a) num[a] += j[s][a] * P.inv_tau[s];
        }
        const R inv_den = R(1) / den;
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            const R tr = P.tau[s] / rho[s];
            const R vx = num[0] * inv_den + tr * F[s][0];
            const R vy = num[1] * inv_den + tr * F[s][1];
            const R vz = num[2] * inv_den + tr * F[s][2];
            const R K = R(1) - R(1.5) * (vx * vx + vy * vy + vz * vz);
            const R wr0 = w0 * rho[s], wr1 = w1 * rho[s], wr2 = w2 * rho[s];
            const R om = P.inv_tau[s];
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const int c = wclass(i);
                const R cv = cdot<LAT, R>(i, vx, vy, vz);
                const R feq = (c == 0 ? wr0 : (c == 1 ? wr1 : wr2)) * (cv * (R(4.5) * cv + R(3)) + K);
                f[s][i] = f[s][i] + om * (feq - f[s][i]);
            }
        }
    }
}

// per-node solute collision; h overwritten with post-collision values
template <int LAT, typename R>
__device__ __forceinline__ void solute_collide(const Phys<R>& P, R (&h)[Lat<LAT>::QS], const R (&u)[3],
                                               R inv_tau) {
    using L = Lat<LAT>;
    R C = 0;
#pragma unroll
    for (int k = 0; k < L::QS; ++k) C += h[k];
#pragma unroll
    for (int k = 0; k < L::QS; ++k) {
        const R W = (k == 0) ? P.Ws0 : P.Ws;
        const R eu = R(L::cx[k]) * u[0] + R(L::cy[k]) * u[1] + R(L::cz[k]) * u[2];
        const R heq = W * C * (R(1) + eu * P.inv_cs2s);
        h[k] = h[k] + inv_tau * (heq - h[k]);
    }
}

template <int LAT, int ST, int NC>
__device__ __forceinline__ void load_shifts(const Phys<typename Store<ST>::R>& P,
                                            typename Store<ST>::R (&sh)[NC][Lat<LAT>::Q]) {
    using R = typename Store<ST>::R;
#pragma unroll
    for (int s = 0; s < NC; ++s)
#pragma unroll
        for (int i = 0; i < Lat<LAT>::Q; ++i) sh[s][i] = (ST >= ST_F16S) ? P.sh[s][i] : R(0);
}

}  // namespace mclbm
