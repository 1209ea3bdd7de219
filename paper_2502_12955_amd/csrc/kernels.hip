// HIP kernels of the multi-component Shan-Chen LBM with reactive solute (gfx950).
//
// A handle holds a batch of independent samples (a single lattice is a batch
// of one).  Storage is fluid-only: the fluid nodes of sample s are numbered
// k = kbase_s .. kbase_s + Nf_s - 1 band by band (bands of y rows, each swept
// plane by plane, row by row, x fastest; kbase_s is a multiple of 64, so no
// 64-node chunk straddles two samples); pos[k] is the
// box index within the sample and map[dbase_s + n] the fluid index (or -1 for
// a solid node).  Populations are kept in chunks of 64 fluid nodes (one
// wavefront): element (plane j, node k) lives at
//   ((k >> 6) * P + j) * 64 + (k & 63),   P = planes of the array,
// so a wavefront reads every plane of its 64 nodes as contiguous rows, and no
// byte of a solid node is moved.  With 16-bit storage of two components the
// flow array pairs the components of each direction in 32-bit words (fidx in
// common.hpp): one load and one store per direction instead of two.  The
// pseudo-potentials follow the fluid numbering, the components of a node
// adjacent (psi[k * NC + s]) so one load fetches both; the collide pass reads
// a neighbour's through the fluid index it also pushes to (a solid neighbour's
// index is -1, and its pseudo-potential counts as 0).
//
// Work distribution: each wavefront processes one chunk at a time, taken from
// a device-side list of active chunks (samples that have converged are left
// out) or from all chunks; the grid is either one pass over the chunks or a
// fixed persistent grid that loops.  Logical blocks are remapped so that each
// XCD (hardware dispatches block b to XCD b % 8) works on a contiguous range
// of chunks, keeping neighbour gathers in one L2.
//
// One step = two kernels, one thread per fluid node:
//   k_density:  rho_s = sum_i f^s_i (eq:1.7), psi_s = rho0 (1 - exp(-rho_s/rho0))
//               (eq:1.11) written at the node's fluid index.
//   k_collide:  forces, velocities, BGK collision with forcing, solute collision,
//               push streaming into buffer B.
// Per fluid node (paper, multi-component LBM section):
//   F^s = -psi_s sum_t G_st sum_i w_i psi_t(x+c_i) c_i          (eq:1.14)
//         -G_ads,s rho_s sum_i w_i s(x+c_i) c_i                  (eq:1.15)
//         +rho_s accel
//   u = (sum_s j_s + F^s/2) / rho                                (eq:1.19)
//   Guo: u^eq_s = u, source eq:1.21 times (1 - 1/(2 tau_s))      (eq:1.16)
//   SC:  u^eq_s = u' + tau_s F^s/rho_s, u' of eq:1.18, no source (eq:1.17)
//   f*_i = f_i + (f^eq_i(rho_s, u^eq_s) - f_i)/tau_s [+ source]   (eq:6, eq:1.16)
// Streaming pushes f*_i to node n + c_i, or back into the node's own slot of
// the opposite direction when n + c_i is solid (halfway bounce-back, eq:5).
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
// Population access of the collide pass, in two addressing forms with the
// same element layout (blk above):
//   GlobalIO: 64-bit flat addresses per element.
//   BufIO:    raw buffer instructions: a 32-bit byte offset per node and
//             the plane offset as a wave-uniform scalar, so a store costs
//             no 64-bit address arithmetic per lane.  Usable while every
//             array is below 4 GiB (the host checks this).
// Both store exactly the same values to the same elements.
// ---------------------------------------------------------------------------
template <int ST, int PF, int HP>
struct GlobalIO {
    using S = Store<ST>;
    using R = typename S::R;
    using T = typename S::T;
    T* __restrict__ fB;
    const T* __restrict__ hA;
    T* __restrict__ hB;
    const T* __restrict__ gA;   // fluid energy populations (GQ planes), conjugate heat transfer only
    T* __restrict__ gB;
    __device__ __forceinline__ void fstore(int j, unsigned kd, R v, R shift) const { S::store(blk(fB, PF, j, kd), v, shift); }
    // paired 16-bit flow storage: both components of direction i (already shifted)
    __device__ __forceinline__ void fstore2(int i, unsigned kd, R v0, R v1) const {
        uint32_t* w = (uint32_t*)fB + ((size_t)(kd >> 6) * (size_t)(PF / 2) + (size_t)i) * 64u + (kd & 63u);
        *w = S::pack2(v0, v1);
    }
    __device__ __forceinline__ R hload(int q, unsigned k) const { return S::load_plain(blk(hA, HP, q, k)); }
    __device__ __forceinline__ void hstore(int q, unsigned kd, R v) const { S::store_plain(blk(hB, HP, q, kd), v); }
    template <int GQ>
    __device__ __forceinline__ R gload(int i, unsigned k) const { return S::load_plain(blk(gA, GQ, i, k)); }
    template <int GQ>
    __device__ __forceinline__ void gstore(int i, unsigned kd, R v) const { S::store_plain(blk(gB, GQ, i, kd), v); }
};

// raw buffer resource: base, no stride, num_records = bytes, gfx9 data format
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

template <int ST>
struct BufBits;
template <>
struct BufBits<ST_F64> {
    template <int AUX>
    __device__ static inline double ld(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
        auto b = __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, AUX);
        uint64_t u = ((uint64_t)b[1] << 32) | b[0];
        return __builtin_bit_cast(double, u);
    }
    __device__ static inline void st(__amdgpu_buffer_rsrc_t r, double v, uint32_t vo, uint32_t so) {
        const uint64_t u = __builtin_bit_cast(uint64_t, v);
        typedef unsigned v2u __attribute__((ext_vector_type(2)));
        v2u b;
        b[0] = (unsigned)u;
        b[1] = (unsigned)(u >> 32);
        __builtin_amdgcn_raw_buffer_store_b64(b, r, vo, so, 0);
    }
};
template <>
struct BufBits<ST_F32> {
    template <int AUX>
    __device__ static inline float ld(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, vo, so, AUX));
    }
    __device__ static inline void st(__amdgpu_buffer_rsrc_t r, float v, uint32_t vo, uint32_t so) {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, vo, so, 0);
    }
};
template <>
struct BufBits<ST_F16S> {
    template <int AUX>
    __device__ static inline float ld(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
        return __half2float(__ushort_as_half(__builtin_amdgcn_raw_buffer_load_b16(r, vo, so, AUX)));
    }
    __device__ static inline void st(__amdgpu_buffer_rsrc_t r, float v, uint32_t vo, uint32_t so) {
        __builtin_amdgcn_raw_buffer_store_b16(__half_as_ushort(__float2half_rn(v)), r, vo, so, 0);
    }
};
template <>
struct BufBits<ST_BF16S> {
    template <int AUX>
    __device__ static inline float ld(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
        return bf16_to_float(__builtin_amdgcn_raw_buffer_load_b16(r, vo, so, AUX));
    }
    __device__ static inline void st(__amdgpu_buffer_rsrc_t r, float v, uint32_t vo, uint32_t so) {
        __builtin_amdgcn_raw_buffer_store_b16(bf16_rne_dev(v), r, vo, so, 0);
    }
};

template <int ST, int PF, int HP>
struct BufIO {
    using S = Store<ST>;
    using R = typename S::R;
    static constexpr uint32_t E = sizeof(typename S::T), PS = 64 * E;   // element and plane bytes
    __amdgpu_buffer_rsrc_t fB, hA, hB, gA, gB;
    // byte offset of (plane 0, node k) in an array of P planes
    template <int P>
    __device__ __forceinline__ static uint32_t node_off(unsigned k) {
        // chunk numbers stay below 2^24 (fluid indices below 2^30), so a 24-bit multiply suffices
        return (__umul24(k >> 6, (uint32_t)(P * 64)) + (k & 63u)) * E;
    }
    __device__ __forceinline__ void fstore(int j, unsigned kd, R v, R shift) const {
        BufBits<ST>::st(fB, v - shift, node_off<PF>(kd) + (uint32_t)j * PS, 0);
    }
    // paired 16-bit flow storage: both components of direction i (already shifted)
    __device__ __forceinline__ void fstore2(int i, unsigned kd, R v0, R v1) const {
        const uint32_t o = (__umul24(kd >> 6, (uint32_t)(PF / 2 * 64)) + (kd & 63u)) * 4u + (uint32_t)i * 256u;
        __builtin_amdgcn_raw_buffer_store_b32(S::pack2(v0, v1), fB, o, 0, 0);
    }
    __device__ __forceinline__ R hload(int q, unsigned k) const {
        return BufBits<ST>::template ld<2>(hA, node_off<HP>(k), (uint32_t)q * PS);
    }
    __device__ __forceinline__ void hstore(int q, unsigned kd, R v) const {
        BufBits<ST>::st(hB, v, node_off<HP>(kd), (uint32_t)q * PS);
    }
    template <int GQ>
    __device__ __forceinline__ R gload(int i, unsigned k) const {
        return BufBits<ST>::template ld<2>(gA, node_off<GQ>(k), (uint32_t)i * PS);
    }
    template <int GQ>
    __device__ __forceinline__ void gstore(int i, unsigned kd, R v) const {
        BufBits<ST>::st(gB, v, node_off<GQ>(kd), (uint32_t)i * PS);
    }
};

struct Geo {
    const SampleDev* smp;
    const int* chunk_sample;
    const unsigned* pos;
    const int* map;
    const uint32_t* links;
    const int* work;   // nullptr: every chunk
    const int* nwork;
    int nchunks;
    int reverse;       // 1: visit the work items in reverse order
};

// Wave-uniform load of a value that no kernel writes while it runs (work
// list, chunk -> sample table, sample records): read through the constant
// address space, so it becomes a scalar load that does not queue behind the
// wavefront's vector loads.
template <class T>
__device__ __forceinline__ T ld_uniform(const T* p) {
    return *(const __attribute__((address_space(4))) T*)p;
}

// Calls body(chunk) for every work item of this wavefront.
template <class Body>
__device__ __forceinline__ void for_each_chunk(const Geo& g, Body body) {
    const int wpb = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int G = gridDim.x;  // multiple of 8
    const int b = blockIdx.x;
    const int lb0 = (b & 7) * (G >> 3) + (b >> 3);
    const int nitems = g.work ? ld_uniform(g.nwork) : g.nchunks;
    for (int it = 0;; ++it) {
        int item = (it * G + lb0) * wpb + wave;
        if (item >= nitems) break;
        if (g.reverse) item = nitems - 1 - item;
        const int ch = g.work ? ld_uniform(g.work + item) : item;
        body(ch);
    }
}

__device__ __forceinline__ SampleDev sample_of(const Geo& g, int ch) {
    const int s = ld_uniform(g.chunk_sample + ch);
    const int* q = (const int*)(g.smp + s);
    SampleDev d;
    d.nx = ld_uniform(q + 0);
    d.ny = ld_uniform(q + 1);
    d.nz = ld_uniform(q + 2);
    d.Nf = ld_uniform(q + 3);
    d.N = ld_uniform(q + 4);
    d.dbase = ld_uniform(q + 5);
    d.kbase = ld_uniform(q + 6);
    d.pad_ = 0;
    return d;
}

// ---------------------------------------------------------------------------
// density / pseudo-potential
// ---------------------------------------------------------------------------
// densities and pseudo-potentials of one 64-node chunk
template <int LAT, int ST, int NC>
__device__ __forceinline__ void density_chunk(const Phys<typename Store<ST>::R>& P, const Geo& g,
                                              const typename Store<ST>::R (&sh)[NC][Lat<LAT>::Q],
                                              const typename Store<ST>::T* __restrict__ fA,
                                              typename Store<ST>::R* __restrict__ psi, int ch) {
    using L = Lat<LAT>;
    using S = Store<ST>;
    using R = typename S::R;
    // populations first: every lane of a chunk is inside the (chunk-padded)
    // arrays, so these loads need not wait for the sample record; tail lanes
    // are discarded below
    const unsigned k = (unsigned)ch * 64u + (threadIdx.x & 63u);
    R rho[NC];
    if constexpr (FlowPairs<ST, NC>::value) {
        const uint32_t* fw = (const uint32_t*)fA + (size_t)(k >> 6) * (L::Q * 64u) + (k & 63u);
        R r0 = 0, r1 = 0;
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            const uint32_t w = __builtin_nontemporal_load(fw + i * 64);
            r0 += S::from_bits(w & 0xffffu) + sh[0][i];
            r1 += S::from_bits(w >> 16) + sh[NC - 1][i];
        }
        rho[0] = r0;
        rho[NC - 1] = r1;
    } else {
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            R r = 0;
#pragma unroll
            for (int i = 0; i < L::Q; ++i) r += S::load(blk(fA, NC * L::Q, s * L::Q + i, k), sh[s][i]);
            rho[s] = r;
        }
    }
    const SampleDev sd = sample_of(g, ch);
    if ((int)(k - (unsigned)sd.kbase) >= sd.Nf) return;
#pragma unroll
    for (int s = 0; s < NC; ++s) psi[(size_t)k * NC + s] = P.rho0 * (R(1) - exp_r<R>(-rho[s] * P.inv_rho0));
}

template <int LAT, int ST, int NC>
__global__ void __launch_bounds__(256) k_density(Phys<typename Store<ST>::R> P, Geo g,
                                                 const typename Store<ST>::T* __restrict__ fA,
                                                 typename Store<ST>::R* __restrict__ psi) {
    using R = typename Store<ST>::R;
    R sh[NC][Lat<LAT>::Q];
    load_shifts<LAT, ST, NC>(P, sh);
    for_each_chunk(g, [&](int ch) { density_chunk<LAT, ST, NC>(P, g, sh, fA, psi, ch); });
}

// ---------------------------------------------------------------------------
// collision of one fluid node and push of its post-collision populations
// (flow with halfway bounce-back; solute with the wet-node reaction, inlet and
// outlet).
//   f: pre-collision flow populations of node k (overwritten)
//   psi_nb(t, d): pseudo-potential of component t of fluid node d (0 for
//                 d = -1, a solid neighbour)
//   dest(i): fluid index of x + c_i, -1 where that node is solid
//   x, nx: x coordinate of the node and the box edge (solute seams)
// ---------------------------------------------------------------------------
template <int LAT, int ST, int NC, int FC, int PR, int KF, int TH, class PsiNb, class Dest, class IO>
__device__ __forceinline__ void collide_push(const Phys<typename Store<ST>::R>& P,
                                             const typename Store<ST>::R (&sh)[NC][Lat<LAT>::Q], unsigned k,
                                             uint32_t lw, int x, int nx, typename Store<ST>::R (&f)[NC][Lat<LAT>::Q],
                                             PsiNb psi_nb, Dest dest, const IO& io) {
    using L = Lat<LAT>;
    using S = Store<ST>;
    using R = typename S::R;
    constexpr int Q = L::Q, QS = L::QS, PF = NC * Q;
    R u[3];
    // fluid indices of the 18 neighbours, gathered together (a solid
    // neighbour reads -1): the pseudo-potential gathers go through them, and
    // the pushes use them without another round trip
    unsigned dst[Q];
    dst[0] = k;
#pragma unroll
    for (int i = 1; i < Q; ++i) dst[i] = dest(i);
    auto psi_d = [&](int t, int i) -> R { return psi_nb(t, dst[i]); };
    flow_collide<LAT, NC, R, decltype(psi_d), FC>(P, lw, f, psi_d, u);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const bool bb = (i != 0) && (lw & (1u << L::opp[i]));
        const unsigned kd = (i != 0 && !bb) ? dst[i] : k;
        const int dir = bb ? L::opp[i] : i;
        if constexpr (FlowPairs<ST, NC>::value) {
            io.fstore2(dir, kd, f[0][i] - sh[0][i], f[NC - 1][i] - sh[NC - 1][i]);  // w_i = w_opp(i)
        } else {
#pragma unroll
            for (int s = 0; s < NC; ++s) io.fstore(s * Q + dir, kd, f[s][i], sh[s][i]);
        }
    }
    if (P.solute) {
        // loaded only now: fewer registers live through the flow part (loading
        // them with the flow populations was measured 0.5 % slower in FP32 and
        // 4 % slower with 16-bit storage)
        R h[QS];
#pragma unroll
        for (int q = 0; q < QS; ++q) h[q] = io.hload(q, k);
        solute_collide<LAT, R>(P, h, u, P.inv_tau_d);
        io.hstore(0, k, h[0]);
        const bool seam_mode = (P.solute == 2);
#pragma unroll
        for (int d = 1; d < QS; ++d) {
            const int dx = L::cx[d];
            const bool seam = seam_mode && ((x == nx - 1 && dx == 1) || (x == 0 && dx == -1));
            if (!seam && !(lw & (1u << L::opp[d]))) {
                const unsigned kd = dst[d];
                io.hstore(d, kd, h[d]);
                if (!TH && (lw & (1u << (L::HOP_SHIFT + d)))) {   // with heat: the interface solve
                    const R Cb = R(2) * h[d] * (KF ? P.kfield[kd] : P.wet_inv_den);
                    io.hstore(L::opp[d], kd, R(2) * P.Ws * Cb - h[d]);
                }
                if (seam_mode && d == L::SXM && x == 1)
                    io.hstore(L::SXP, kd, R(2) * P.Ws * P.C_in - h[d]);
            }
            if (seam_mode && d == L::SXM && x == nx - 1) io.hstore(d, k, h[d]);
        }
        if (PR) {
            // the product (planes QS..2QS-1): same collision with its own tau, same
            // streaming; a reacting link creates k C_b of it (C_b of the reacting
            // species on that link, from h[d] above), entering in its own flux
            // convention: h2_out = h2_in + k tau2 / (tau2 - 1/2) C_b
            R h2[QS];
#pragma unroll
            for (int q = 0; q < QS; ++q) h2[q] = io.hload(QS + q, k);
            solute_collide<LAT, R>(P, h2, u, P.inv_tau_d2);
            io.hstore(QS, k, h2[0]);
#pragma unroll
            for (int d = 1; d < QS; ++d) {
                const int dx = L::cx[d];
                const bool seam = seam_mode && ((x == nx - 1 && dx == 1) || (x == 0 && dx == -1));
                if (!seam && !(lw & (1u << L::opp[d]))) {
                    const unsigned kd = dst[d];
                    io.hstore(QS + d, kd, h2[d]);
                    if (!TH && (lw & (1u << (L::HOP_SHIFT + d)))) {
                        const R Cb = R(2) * h[d] * (KF ? P.kfield[kd] : P.wet_inv_den);
                        const R gain = KF ? P.kfield[P.kstride + kd] : P.prod_gain;
                        io.hstore(QS + L::opp[d], kd, h2[d] + gain * Cb);
                    }
                    if (seam_mode && d == L::SXM && x == 1)
                        io.hstore(QS + L::SXP, kd, R(2) * P.Ws * P.C_in2 - h2[d]);
                }
                if (seam_mode && d == L::SXM && x == nx - 1) io.hstore(QS + d, k, h2[d]);
            }
        }
    }
    if (TH) {
        // fluid energy populations (eq:therpop, eq:therpopeq): BGK towards
        // w_i E [1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u.u], E = sum g, with the
        // barycentric velocity; pushed to fluid neighbours only (a population
        // heading into a solid leaves the fluid; the interface solve supplies
        // the ones arriving from solids)
        R g[Q];
        R E = 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            g[i] = io.template gload<Q>(i, k);
            E += g[i];
        }
        const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const R cu = cdot<LAT, R>(i, u[0], u[1], u[2]);
            const R geq = wgt<LAT, R>(i) * E * (R(1) + R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu);
            const R post = g[i] - (g[i] - geq) * P.th_inv_tau_ef;
            if (i == 0)
                io.template gstore<Q>(0, k, post);
            else if (!(lw & (1u << L::opp[i])))
                io.template gstore<Q>(i, dst[i], post);
        }
    }
}

// ---------------------------------------------------------------------------
// collision + push streaming
// ---------------------------------------------------------------------------
// collision and push of one 64-node chunk
template <int LAT, int ST, int NC, int FC, int SV, int BUF>
__device__ __forceinline__ void collide_chunk(const Phys<typename Store<ST>::R>& P, const Geo& g,
                                              const typename Store<ST>::R (&sh)[NC][Lat<LAT>::Q],
                                              const typename Store<ST>::T* __restrict__ fA,
                                              typename Store<ST>::T* __restrict__ fB,
                                              const typename Store<ST>::T* __restrict__ hA,
                                              typename Store<ST>::T* __restrict__ hB,
                                              const typename Store<ST>::R* __restrict__ psi, uint32_t fbytes,
                                              uint32_t hbytes, const typename Store<ST>::T* __restrict__ gA,
                                              typename Store<ST>::T* __restrict__ gB, uint32_t gbytes,
                                              uint32_t pbytes, int ch) {
    using L = Lat<LAT>;
    using S = Store<ST>;
    using R = typename S::R;
    constexpr int Q = L::Q, PF = NC * Q, QS = L::QS, HP = QS * (1 + (SV & 1));
    // No tail check: the lanes past a sample's last fluid node (up to the
    // 64-node chunk boundary) carry pos 0 and a link word with every flow
    // link blocked, so they read inside the sample and store only into
    // their own (unused) slots.  Node-local loads are issued first.
    const unsigned k = (unsigned)ch * 64u + (threadIdx.x & 63u);
    // read once per step, like the populations: non-temporal, so they do not
    // displace the neighbour indices and pseudo-potentials that other nodes gather
    const unsigned n = __builtin_nontemporal_load(g.pos + k);
    const uint32_t lw = __builtin_nontemporal_load(g.links + k);
    R f[NC][Q];
    if constexpr (FlowPairs<ST, NC>::value) {
        // both components of direction i in one 32-bit word
        uint32_t w[Q];
        if constexpr (BUF) {
            const __amdgpu_buffer_rsrc_t fr = make_rsrc(fA, fbytes);
            const uint32_t vo = (__umul24(k >> 6, (uint32_t)(Q * 64)) + (k & 63u)) * 4u;
#pragma unroll
            for (int i = 0; i < Q; ++i) w[i] = __builtin_amdgcn_raw_buffer_load_b32(fr, vo, (uint32_t)i * 256u, 2);
        } else {
            const uint32_t* fw = (const uint32_t*)fA + (size_t)(k >> 6) * (Q * 64u) + (k & 63u);
#pragma unroll
            for (int i = 0; i < Q; ++i) w[i] = __builtin_nontemporal_load(fw + i * 64);
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            f[0][i] = S::from_bits(w[i] & 0xffffu) + sh[0][i];
            f[NC - 1][i] = S::from_bits(w[i] >> 16) + sh[NC - 1][i];
        }
    } else if constexpr (BUF) {
        const __amdgpu_buffer_rsrc_t fr = make_rsrc(fA, fbytes);
        const uint32_t vo = BufIO<ST, PF, HP>::template node_off<PF>(k);
#pragma unroll
        for (int s = 0; s < NC; ++s)
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const R v = BufBits<ST>::template ld<2>(fr, vo, (uint32_t)(s * Q + i) * BufIO<ST, PF, HP>::PS);
                f[s][i] = (ST >= ST_F16S) ? v + sh[s][i] : v;
            }
    } else {
#pragma unroll
        for (int s = 0; s < NC; ++s)
#pragma unroll
            for (int i = 0; i < Q; ++i) f[s][i] = S::load(blk(fA, PF, s * Q + i, k), sh[s][i]);
    }
    const SampleDev sd = sample_of(g, ch);
    int x, y, z;
    coords(n, sd.nx, sd.ny, x, y, z);
    const NbIdx nb = make_nb(x, y, z, sd.nx, sd.ny, sd.nz);
    const int* mp = g.map + sd.dbase;
    if constexpr (BUF) {
        const __amdgpu_buffer_rsrc_t mr = make_rsrc(mp, (uint32_t)sd.N * 4u);
        const __amdgpu_buffer_rsrc_t pr = make_rsrc(psi, pbytes);
        // d = -1 gives a byte offset of at least 2^32 - 16 (32-bit wrap), past
        // the record size (a multiple of 256 below 2^32), and a raw buffer load
        // outside the record returns 0: the solid neighbour's value
        auto psi_nb = [&](int t, unsigned d) -> R {
            const uint32_t o = d * (uint32_t)(NC * sizeof(R)) + t * sizeof(R);
            if constexpr (sizeof(R) == 8) return BufBits<ST_F64>::template ld<0>(pr, o, 0);
            else return BufBits<ST_F32>::template ld<0>(pr, o, 0);
        };
        auto dest = [&](int i) -> unsigned {
            return __builtin_amdgcn_raw_buffer_load_b32(mr, nb.at(L::cx[i], L::cy[i], L::cz[i]) * 4u, 0, 0);
        };
        BufIO<ST, PF, HP> io;
        io.fB = make_rsrc(fB, fbytes);
        io.hA = make_rsrc(hA, hbytes);
        io.hB = make_rsrc(hB, hbytes);
        io.gA = make_rsrc(gA, gbytes);
        io.gB = make_rsrc(gB, gbytes);
        collide_push<LAT, ST, NC, FC, (SV & 1), ((SV >> 1) & 1), (SV >> 2)>(P, sh, k, lw, x, sd.nx, f, psi_nb, dest,
                                                                              io);
    } else {
        auto psi_nb = [&](int t, unsigned d) -> R { return d == ~0u ? R(0) : psi[(size_t)d * NC + t]; };
        auto dest = [&](int i) -> unsigned { return (unsigned)mp[nb.at(L::cx[i], L::cy[i], L::cz[i])]; };
        const GlobalIO<ST, PF, HP> io{fB, hA, hB, gA, gB};
        collide_push<LAT, ST, NC, FC, (SV & 1), ((SV >> 1) & 1), (SV >> 2)>(P, sh, k, lw, x, sd.nx, f, psi_nb, dest,
                                                                              io);
    }
}

// FC: forcing scheme (0 Guo, 1 Shan-Chen); SV: solute variant, bit 0 the
// product species, bit 1 the per-node rate field, bit 2 conjugate heat transfer
// (each compiled in or out, so the plain path keeps its registers and
// schedule); BUF: buffer addressing (BufIO, every array below 4 GiB) or flat
// addresses (GlobalIO)
template <int LAT, int ST, int NC, int FC, int SV, int BUF>
__global__ void __launch_bounds__(256) k_collide(Phys<typename Store<ST>::R> P, Geo g,
                                                 const typename Store<ST>::T* __restrict__ fA,
                                                 typename Store<ST>::T* __restrict__ fB,
                                                 const typename Store<ST>::T* __restrict__ hA,
                                                 typename Store<ST>::T* __restrict__ hB,
                                                 const typename Store<ST>::R* __restrict__ psi,
                                                 uint32_t fbytes, uint32_t hbytes,
                                                 const typename Store<ST>::T* __restrict__ gA,
                                                 typename Store<ST>::T* __restrict__ gB, uint32_t gbytes,
                                                 uint32_t pbytes) {
    using R = typename Store<ST>::R;
    R sh[NC][Lat<LAT>::Q];
    load_shifts<LAT, ST, NC>(P, sh);
    for_each_chunk(g, [&](int ch) {
        collide_chunk<LAT, ST, NC, FC, SV, BUF>(P, g, sh, fA, fB, hA, hB, psi, fbytes, hbytes, gA, gB, gbytes, pbytes,
                                                ch);
    });
}

// ---------------------------------------------------------------------------
// initialisation at equilibrium (no force term) from dense staging fields
// laid out per sample: rho [nc][N_s], u [3][N_s], C [N_s], samples concatenated
// ---------------------------------------------------------------------------
template <int LAT, int ST, int NC>
__global__ void __launch_bounds__(256) k_init_eq(Phys<typename Store<ST>::R> P, Geo g,
                                                 typename Store<ST>::T* __restrict__ fA,
                                                 typename Store<ST>::T* __restrict__ hA,
                                                 const double* __restrict__ rho, const double* __restrict__ u,
                                                 const double* __restrict__ C) {
    using L = Lat<LAT>;
    using S = Store<ST>;
    using R = typename S::R;
    R sh[NC][L::Q];
    load_shifts<LAT, ST, NC>(P, sh);
    for_each_chunk(g, [&](int ch) {
        const SampleDev sd = sample_of(g, ch);
        const unsigned k = (unsigned)ch * 64u + (threadIdx.x & 63u);
        if ((int)(k - (unsigned)sd.kbase) >= sd.Nf) return;
        const size_t N = sd.N;
        const unsigned n = g.pos[k];
        R v[3] = {0, 0, 0};
        if (u) {
            const double* us = u + (size_t)3 * sd.dbase;
            v[0] = (R)us[n];
            v[1] = (R)us[N + n];
            v[2] = (R)us[2 * N + n];
        }
        const R vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        const double* rs = rho + (size_t)NC * sd.dbase;
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            const R r = (R)rs[s * N + n];
#pragma unroll
            for (int i = 0; i < L::Q; ++i) {
                const R cv = R(L::cx[i]) * v[0] + R(L::cy[i]) * v[1] + R(L::cz[i]) * v[2];
                const R feq = wgt<LAT, R>(i) * r * (R(1) + R(3) * cv + R(4.5) * cv * cv - R(1.5) * vv);
                S::store(fA + fidx<ST, NC, L::Q>(s * L::Q + i, k), feq, sh[s][i]);
            }
        }
        if (P.solute) {
            const R c0 = C ? (R)C[(size_t)sd.dbase + n] : R(0);
#pragma unroll
            for (int q = 0; q < L::QS; ++q) {
                const R W = (q == 0) ? P.Ws0 : P.Ws;
                const R eu = R(L::cx[q]) * v[0] + R(L::cy[q]) * v[1] + R(L::cz[q]) * v[2];
                S::store_plain(blk(hA, P.hplanes, q, k), W * c0 * (R(1) + eu * P.inv_cs2s));
            }
            if (P.product)   // no product at t = 0
                for (int q = 0; q < L::QS; ++q) S::store_plain(blk(hA, P.hplanes, L::QS + q, k), R(0));
        }
    });
}

// ---------------------------------------------------------------------------
// moments of the current state: rho_s, barycentric u with half force, C.
// Reuses flow_collide for the force and velocity (the post-collision values
// it leaves in the local copy are discarded).
// ---------------------------------------------------------------------------
template <int LAT, int ST, int NC>
__device__ __forceinline__ void node_moments(const Phys<typename Store<ST>::R>& P, const Geo& g,
                                             const SampleDev& sd, unsigned k,
                                             const typename Store<ST>::T* __restrict__ fA,
                                             const typename Store<ST>::T* __restrict__ hA,
                                             const typename Store<ST>::R* __restrict__ psi,
                                             typename Store<ST>::R (&rho)[NC], typename Store<ST>::R (&u)[3],
                                             typename Store<ST>::R& C, typename Store<ST>::R& C2) {
    using L = Lat<LAT>;
    using S = Store<ST>;
    using R = typename S::R;
    R sh[NC][L::Q];
    load_shifts<LAT, ST, NC>(P, sh);
    const unsigned n = g.pos[k];
    const uint32_t lw = g.links[k];
    int x, y, z;
    coords(n, sd.nx, sd.ny, x, y, z);
    const NbIdx nb = make_nb(x, y, z, sd.nx, sd.ny, sd.nz);
    const int* mp = g.map + sd.dbase;
    R f[NC][L::Q];
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        R r = 0;
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            f[s][i] = S::load(fA + fidx<ST, NC, L::Q>(s * L::Q + i, k), sh[s][i]);
            r += f[s][i];
        }
        rho[s] = r;
    }
    auto psi_nb = [&](int t, int i) -> R {
        const int d = mp[nb.at(L::cx[i], L::cy[i], L::cz[i])];
        return d < 0 ? R(0) : psi[(size_t)d * NC + t];
    };
    flow_collide<LAT, NC, R>(P, lw, f, psi_nb, u);
    C = 0;
    C2 = 0;
    if (P.solute) {
#pragma unroll
        for (int q = 0; q < L::QS; ++q) C += S::load_plain(blk(hA, P.hplanes, q, k));
        if (P.product)
            for (int q = 0; q < L::QS; ++q) C2 += S::load_plain(blk(hA, P.hplanes, L::QS + q, k));
    }
}

__global__ void __launch_bounds__(256) k_fill(double* __restrict__ p, long long n, double v) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

template <int LAT, int ST, int NC>
__global__ void __launch_bounds__(256) k_moments_out(Phys<typename Store<ST>::R> P, Geo g,
                                                     const typename Store<ST>::T* __restrict__ fA,
                                                     const typename Store<ST>::T* __restrict__ hA,
                                                     const typename Store<ST>::R* __restrict__ psi,
                                                     double* __restrict__ rho_out, double* __restrict__ u_out,
                                                     double* __restrict__ C_out) {
    using R = typename Store<ST>::R;
    for_each_chunk(g, [&](int ch) {
        const SampleDev sd = sample_of(g, ch);
        const unsigned k = (unsigned)ch * 64u + (threadIdx.x & 63u);
        if ((int)(k - (unsigned)sd.kbase) >= sd.Nf) return;
        R rho[NC], u[3], C, C2;
        node_moments<LAT, ST, NC>(P, g, sd, k, fA, hA, psi, rho, u, C, C2);
        const size_t N = sd.N;
        const unsigned n = g.pos[k];
        if (rho_out)
            for (int s = 0; s < NC; ++s) rho_out[(size_t)NC * sd.dbase + s * N + n] = (double)rho[s];
        if (u_out)
            for (int a = 0; a < 3; ++a) u_out[(size_t)3 * sd.dbase + a * N + n] = (double)u[a];
        if (C_out) {
            // [species][N] per sample block: the product follows the reacting species
            const int nsp = P.product ? 2 : 1;
            C_out[(size_t)nsp * sd.dbase + n] = (double)C;
            if (P.product) C_out[(size_t)2 * sd.dbase + N + n] = (double)C2;
        }
    });
}

// ---------------------------------------------------------------------------
// encoding of caller-supplied FP64 populations into the storage format, with
// the same store the step kernels use: elements q0 .. q0 + cnt - 1 of a
// chunked array of P planes (a flow array in its own layout, fidx); in a flow
// array (flow = 1) plane j is component j / Q, direction j % Q and carries the
// storage shift of that pair; solute planes are stored unshifted.  The value
// is rounded to the arithmetic type first, then shifted and rounded to the
// stored type.
// ---------------------------------------------------------------------------
template <int LAT, int ST, int NC>
__global__ void __launch_bounds__(256) k_encode(Phys<typename Store<ST>::R> P, const double* __restrict__ src,
                                                typename Store<ST>::T* __restrict__ dst, long long q0, long long cnt,
                                                int planes, int flow) {
    using S = Store<ST>;
    using R = typename S::R;
    constexpr int Q = Lat<LAT>::Q;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt) return;
    const long long q = q0 + t;
    const R v = (R)src[t];
    if (flow) {
        int s, i;
        if constexpr (FlowPairs<ST, NC>::value) {
            const int r = (int)(q % (Q * 128));   // element within its chunk: (i, node, s)
            i = r >> 7;
            s = r & 1;
        } else {
            const int j = (int)((q >> 6) % planes);
            s = j / Q;
            i = j % Q;
        }
        S::store(dst + q, v, (ST >= ST_F16S) ? P.sh[s][i] : R(0));
    } else {
        S::store_plain(dst + q, v);
    }
}

// ---------------------------------------------------------------------------
// particle deposition (sec:particle_deposition, eq:surface_deposition): after
// a step, every fluid node with a solid flow-lattice neighbour adds DP times
// its particle concentration (the reacting solute species: the sum of its
// populations after streaming, in FP64) to its deposit.  Nodes whose deposit
// then exceeds 1 are counted; the host turns them solid.
// ---------------------------------------------------------------------------
template <int LAT, int ST>
__global__ void __launch_bounds__(256) k_deposit(Phys<typename Store<ST>::R> P, Geo g,
                                                 const typename Store<ST>::T* __restrict__ hA,
                                                 double* __restrict__ dep, double DP, int* __restrict__ count) {
    using L = Lat<LAT>;
    using S = Store<ST>;
    for_each_chunk(g, [&](int ch) {
        const SampleDev sd = sample_of(g, ch);
        const unsigned k = (unsigned)ch * 64u + (threadIdx.x & 63u);
        if ((int)(k - (unsigned)sd.kbase) >= sd.Nf) return;
        const uint32_t lw = g.links[k];
        if ((lw & ((1u << L::Q) - 2u)) == 0u) return;   // no solid neighbour
        double C = 0.0;
#pragma unroll
        for (int q = 0; q < L::QS; ++q) C += (double)S::load_plain(blk(hA, P.hplanes, q, k));
        const double d = dep[k] + DP * C;
        dep[k] = d;
        if (d > 1.0) atomicAdd(count, 1);
    });
}

// ---------------------------------------------------------------------------
// monitors: FP64 per-chunk partials (one wavefront each), then a fixed-order
// reduction per sample.
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
__global__ void __launch_bounds__(256) k_monitor(Phys<typename Store<ST>::R> P, Geo g,
                                                 const typename Store<ST>::T* __restrict__ fA,
                                                 const typename Store<ST>::T* __restrict__ hA,
                                                 const typename Store<ST>::R* __restrict__ psi,
                                                 typename Store<ST>::R* __restrict__ snap, size_t M,
                                                 int have_snapshot, double* __restrict__ partials) {
    using R = typename Store<ST>::R;
    for_each_chunk(g, [&](int ch) {
        const SampleDev sd = sample_of(g, ch);
        const unsigned k = (unsigned)ch * 64u + (threadIdx.x & 63u);
        double v[MON_NV];
#pragma unroll
        for (int q = 0; q < MON_NV; ++q) v[q] = 0.0;
        if ((int)(k - (unsigned)sd.kbase) < sd.Nf) {
            R rho[NC], u[3], C;
            R C2;
            node_moments<LAT, ST, NC>(P, g, sd, k, fA, hA, psi, rho, u, C, C2);
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
                    const double d = ua - (double)snap[a * M + k];
                    du += d * d;
                }
                snap[a * M + k] = u[a];
            }
            v[3] = du;
            v[4] = uu;
            if (have_snapshot) {
                const double dp = (double)phi - (double)snap[3 * M + k];
                const double dc = (double)C - (double)snap[4 * M + k];
                v[5] = dp * dp;
                v[7] = dc * dc;
            }
            v[6] = (double)phi * (double)phi;
            v[8] = (double)C * (double)C;
            snap[3 * M + k] = phi;
            snap[4 * M + k] = C;
            const bool bad = !isfinite((double)rho[0]) || !isfinite((double)rho[NC - 1]) || !isfinite((double)C) ||
                             !isfinite((double)u[0]) || !isfinite((double)u[1]) || !isfinite((double)u[2]);
            v[9] = bad ? 1.0 : 0.0;
            v[10] = 1.0;
        }
#pragma unroll
        for (int q = 0; q < MON_NV; ++q) {
            const double s = wave_sum(v[q]);
            if ((threadIdx.x & 63) == 0) partials[(size_t)ch * MON_NV + q] = s;
        }
    });
}

// one block of 256 threads per sample: thread t sums the sample's chunks
// t, t+256, ... in order, then a fixed tree over the 256 threads
__global__ void __launch_bounds__(256) k_monitor_final(const double* __restrict__ partials,
                                                       const SampleDev* __restrict__ smp,
                                                       double* __restrict__ result) {
    __shared__ double acc[256][MON_NV + 1];
    const SampleDev sd = smp[blockIdx.x];
    const long long c0 = sd.kbase >> 6, nch = (sd.Nf + 63) >> 6;
    const int t = threadIdx.x;
    double s[MON_NV];
#pragma unroll
    for (int q = 0; q < MON_NV; ++q) s[q] = 0.0;
    for (long long b = t; b < nch; b += 256)
#pragma unroll
        for (int q = 0; q < MON_NV; ++q) s[q] += partials[(c0 + b) * MON_NV + q];
#pragma unroll
    for (int q = 0; q < MON_NV; ++q) acc[t][q] = s[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
#pragma unroll
            for (int q = 0; q < MON_NV; ++q) acc[t][q] += acc[t + w][q];
        __syncthreads();
    }
    if (t < MON_NV) result[(size_t)blockIdx.x * 16 + t] = acc[0][t];
}

// ---------------------------------------------------------------------------
// host dispatch
// ---------------------------------------------------------------------------
float shift_f32(const Ctx& c, int s, int i) {
    if (c.st < ST_F16S) return 0.0f;
    static const int wn19[19] = {12, 2, 2, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
    static const int wn9[9] = {16, 4, 4, 4, 4, 1, 1, 1, 1};
    if (i >= ((c.lat == 1) ? 19 : 9)) return 0.0f;
    const int wn = (c.lat == 1) ? wn19[i] : wn9[i];
    const float w = (float)wn / 36.0f;
    return w * (float)c.rhobar[s];
}

template <typename R>
Phys<R> make_phys(const Ctx& c) {
    Phys<R> P;
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
    P.product = c.product;
    P.hplanes = c.hplanes;
    const double tau_d2 = (c.D2 > 0 ? c.D2 : 1.0) / cs2s + 0.5;
    P.inv_tau_d2 = (R)(1.0 / tau_d2);
    P.prod_gain = (R)(c.k_wall * tau_d2 / (tau_d2 - 0.5));
    P.C_in2 = (R)c.C_in2;
    P.kfield = (const R*)c.kfield;
    P.kstride = (unsigned)(c.nchunks * 64);
    P.th_inv_tau_ef = (R)(c.thermal ? 1.0 / c.th_tau_ef : 1.0);
    return P;
}
template Phys<float> make_phys<float>(const Ctx&);
template Phys<double> make_phys<double>(const Ctx&);

template <int ST>
using SR = typename Store<ST>::R;
template <int ST>
using STT = typename Store<ST>::T;

static inline Geo make_geo(const Ctx& c, bool use_work) {
    Geo g;
    g.smp = c.smp;
    g.chunk_sample = c.chunk_sample;
    g.pos = c.pos;
    g.map = c.map;
    g.links = c.links;
    g.work = use_work ? c.work : nullptr;
    g.nwork = c.nwork;
    g.nchunks = (int)c.nchunks;
    g.reverse = 0;
    return g;
}

// grid: blocks of bs threads (bs/64 chunks per pass), multiple of 8 for the XCD remap
// (sized for the active chunks when a work list is in use; a smaller grid than
// the items only makes the wavefronts loop)
static inline dim3 grid_for(const Ctx& c, int bs, bool persistent) {
    const long long wpb = bs / 64;
    const long long items = c.work ? c.nactive : c.nchunks;
    long long nb = (items + wpb - 1) / wpb;
    if (persistent && c.grid > 0 && c.grid < nb) nb = c.grid;
    nb = (nb + 7) & ~7LL;
    return dim3((unsigned)(nb > 0 ? nb : 8));
}

template <int LAT, int ST, int NC>
static hipError_t step_t(const Ctx& c) {
    auto P = make_phys<SR<ST>>(c);
    const Geo g = make_geo(c, true);
    const int bs = c.block > 0 ? c.block : 256;
    const dim3 grid = grid_for(c, bs, true);

    // the collide pass walks the chunks in the opposite order of the density
    // pass, so it starts on the chunks the density pass read last
    Geo gr = g;
    gr.reverse = 1;
    const STT<ST>* fA = (const STT<ST>*)c.fA;
    STT<ST>* fB = (STT<ST>*)c.fB;
    const STT<ST>* hA = (const STT<ST>*)c.hA;
    STT<ST>* hB = (STT<ST>*)c.hB;
    const SR<ST>* psi = (const SR<ST>*)c.psi;
    // buffer addressing needs every population array, the pseudo-potentials
    // and each sample's map below 4 GiB (32-bit byte offsets)
    const size_t fbytes = (size_t)c.nchunks * 64 * NC * Lat<LAT>::Q * sizeof(STT<ST>);
    const size_t pbytes = (size_t)c.nchunks * 64 * NC * sizeof(SR<ST>);
    const size_t hbytes = (size_t)c.nchunks * 64 * (size_t)(c.hplanes > 0 ? c.hplanes : 1) * sizeof(STT<ST>);
    const size_t gbytes = c.thermal ? (size_t)c.nchunks * 64 * Lat<LAT>::Q * sizeof(STT<ST>) : 0;
    const bool buf = !c.flat && fbytes < (1ull << 32) && hbytes < (1ull << 32) && gbytes < (1ull << 32) &&
                     pbytes < (1ull << 32) && (size_t)c.max_sample_nodes * 4 < (1ull << 32);
    const uint32_t fb32 = (uint32_t)(buf ? fbytes : 0), hb32 = (uint32_t)(buf ? hbytes : 0),
                   gb32 = (uint32_t)(buf ? gbytes : 0), pb32 = (uint32_t)(buf ? pbytes : 0);
    const STT<ST>* gA = (const STT<ST>*)c.gA;
    STT<ST>* gB = (STT<ST>*)c.gB;
    hipLaunchKernelGGL((k_density<LAT, ST, NC>), grid, dim3(bs), 0, c.stream, P, g, (const STT<ST>*)c.fA,
                       (SR<ST>*)c.psi);
#define MCLBM_COLLIDE(FC, SV)                                                                                    \
    do {                                                                                                         \
        if (buf)                                                                                                 \
            hipLaunchKernelGGL((k_collide<LAT, ST, NC, FC, SV, 1>), grid, dim3(bs), 0, c.stream, P, gr, fA, fB, \
                               hA, hB, psi, fb32, hb32, gA, gB, gb32, pb32);                                     \
        else                                                                                                     \
            hipLaunchKernelGGL((k_collide<LAT, ST, NC, FC, SV, 0>), grid, dim3(bs), 0, c.stream, P, gr, fA, fB, \
                               hA, hB, psi, fb32, hb32, gA, gB, gb32, pb32);                                     \
    } while (0)
    if (c.thermal) {
        // conjugate heat transfer (F64 / F32 storage, uniform rate law of T):
        // SV bit 2 on, then the solid energy pass and the interface solve
        if constexpr (ST <= ST_F32) {
            switch (c.forcing * 2 + (c.product ? 1 : 0)) {
                case 0: MCLBM_COLLIDE(0, 4); break;
                case 1: MCLBM_COLLIDE(0, 5); break;
                case 2: MCLBM_COLLIDE(1, 4); break;
                default: MCLBM_COLLIDE(1, 5); break;
            }
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            return k_thermal_step(c);
        } else {
            return hipErrorInvalidValue;
        }
    }
    const int sv = (c.product ? 1 : 0) + (c.kfield ? 2 : 0);
    switch (c.forcing * 4 + sv) {
        case 0: MCLBM_COLLIDE(0, 0); break;
        case 1: MCLBM_COLLIDE(0, 1); break;
        case 2: MCLBM_COLLIDE(0, 2); break;
        case 3: MCLBM_COLLIDE(0, 3); break;
        case 4: MCLBM_COLLIDE(1, 0); break;
        case 5: MCLBM_COLLIDE(1, 1); break;
        case 6: MCLBM_COLLIDE(1, 2); break;
        default: MCLBM_COLLIDE(1, 3); break;
    }
#undef MCLBM_COLLIDE
    return hipGetLastError();
}

template <int LAT, int ST, int NC>
static hipError_t init_t(const Ctx& c, const double* rho, const double* u, const double* C) {
    auto P = make_phys<SR<ST>>(c);
    const Geo g = make_geo(c, false);
    hipLaunchKernelGGL((k_init_eq<LAT, ST, NC>), grid_for(c, 256, false), dim3(256), 0, c.stream, P, g,
                       (STT<ST>*)c.fA, (STT<ST>*)c.hA, rho, u, C);
    return hipGetLastError();
}

template <int LAT, int ST, int NC>
static hipError_t moments_t(const Ctx& c, double* rho, double* u, double* C) {
    auto P = make_phys<SR<ST>>(c);
    const Geo g = make_geo(c, false);
    const dim3 grid = grid_for(c, 256, false);
    auto fill = [&](double* p, long long n) {
        if (p) hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c.stream, p, n, 0.0);
    };
    fill(rho, (long long)NC * c.Ntot);
    fill(u, 3LL * c.Ntot);
    fill(C, (1LL + c.product) * c.Ntot);   // one plane per solute species; solid nodes stay 0
    hipLaunchKernelGGL((k_density<LAT, ST, NC>), grid, dim3(256), 0, c.stream, P, g, (const STT<ST>*)c.fA,
                       (SR<ST>*)c.psi);
    hipLaunchKernelGGL((k_moments_out<LAT, ST, NC>), grid, dim3(256), 0, c.stream, P, g, (const STT<ST>*)c.fA,
                       (const STT<ST>*)c.hA, (const SR<ST>*)c.psi, rho, u, C);
    return hipGetLastError();
}

template <int LAT, int ST, int NC>
static hipError_t monitor_t(const Ctx& c, int have_snapshot) {
    auto P = make_phys<SR<ST>>(c);
    const Geo g = make_geo(c, true);
    const dim3 grid = grid_for(c, 256, true);
    hipLaunchKernelGGL((k_density<LAT, ST, NC>), grid, dim3(256), 0, c.stream, P, g, (const STT<ST>*)c.fA,
                       (SR<ST>*)c.psi);
    hipLaunchKernelGGL((k_monitor<LAT, ST, NC>), grid, dim3(256), 0, c.stream, P, g, (const STT<ST>*)c.fA,
                       (const STT<ST>*)c.hA, (const SR<ST>*)c.psi, (SR<ST>*)c.snap, (size_t)c.nchunks * 64,
                       have_snapshot, c.partials);
    hipLaunchKernelGGL(k_monitor_final, dim3(c.nsamples), dim3(256), 0, c.stream, (const double*)c.partials, c.smp,
                       c.result);
    return hipGetLastError();
}

template <int LAT, int ST, int NC>
static hipError_t deposit_t(const Ctx& c, double* dep, double DP, int* count) {
    auto P = make_phys<SR<ST>>(c);
    const Geo g = make_geo(c, false);
    hipLaunchKernelGGL((k_deposit<LAT, ST>), grid_for(c, 256, false), dim3(256), 0, c.stream, P, g,
                       (const STT<ST>*)c.hA, dep, DP, count);
    return hipGetLastError();
}

template <int LAT, int ST, int NC>
static hipError_t encode_t(const Ctx& c, const double* src, void* dst, long long q0, long long cnt, int planes,
                           int flow) {
    if (cnt <= 0) return hipSuccess;
    auto P = make_phys<SR<ST>>(c);
    hipLaunchKernelGGL((k_encode<LAT, ST, NC>), dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, c.stream, P, src,
                       (STT<ST>*)dst, q0, cnt, planes, flow);
    return hipGetLastError();
}

#define MCLBM_DISPATCH(FN, ...)                                \
    do {                                                       \
        const int key = c.lat * 100 + c.st * 10 + c.nc;        \
        switch (key) {                                         \
            case 1: return FN<0, 0, 1>(__VA_ARGS__);           \
            case 2: return FN<0, 0, 2>(__VA_ARGS__);           \
            case 11: return FN<0, 1, 1>(__VA_ARGS__);          \
            case 12: return FN<0, 1, 2>(__VA_ARGS__);          \
            case 21: return FN<0, 2, 1>(__VA_ARGS__);          \
            case 22: return FN<0, 2, 2>(__VA_ARGS__);          \
            case 31: return FN<0, 3, 1>(__VA_ARGS__);          \
            case 32: return FN<0, 3, 2>(__VA_ARGS__);          \
            case 101: return FN<1, 0, 1>(__VA_ARGS__);         \
            case 102: return FN<1, 0, 2>(__VA_ARGS__);         \
            case 111: return FN<1, 1, 1>(__VA_ARGS__);         \
            case 112: return FN<1, 1, 2>(__VA_ARGS__);         \
            case 121: return FN<1, 2, 1>(__VA_ARGS__);         \
            case 122: return FN<1, 2, 2>(__VA_ARGS__);         \
            case 131: return FN<1, 3, 1>(__VA_ARGS__);         \
            case 132: return FN<1, 3, 2>(__VA_ARGS__);         \
            default: return hipErrorInvalidValue;              \
        }                                                      \
    } while (0)

hipError_t k_init(const Ctx& c, const double* rho, const double* u, const double* C) {
    MCLBM_DISPATCH(init_t, c, rho, u, C);
}
hipError_t k_step(const Ctx& c) { MCLBM_DISPATCH(step_t, c); }
hipError_t k_moments(const Ctx& c, double* rho, double* u, double* C) { MCLBM_DISPATCH(moments_t, c, rho, u, C); }
hipError_t k_monitor(const Ctx& c, int have_snapshot) { MCLBM_DISPATCH(monitor_t, c, have_snapshot); }
hipError_t k_encode_planes(const Ctx& c, const double* src, void* dst, long long q0, long long cnt, int planes,
                          int flow) {
    MCLBM_DISPATCH(encode_t, c, src, dst, q0, cnt, planes, flow);
}
hipError_t k_deposit_step(const Ctx& c, double* dep, double DP, int* count) {
    MCLBM_DISPATCH(deposit_t, c, dep, DP, count);
}

}  // namespace mclbm
