// Shared device-side definitions: lattice traits, storage policies, kernel
// arguments and the per-node link word.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mclbm {

// ---------------------------------------------------------------------------
// Lattices.  Velocity order follows the paper's tables ("3D and 2D LBM
// Models"): D3Q19 and D2Q9 (w_4 = 1/9).  The solute lattice takes the first
// QS vectors of the flow lattice (D3Q7 / D2Q5), so a solute direction k and
// the flow direction k point the same way.  Flow weights are wn[i] / 36.
// ---------------------------------------------------------------------------
template <int LAT>
struct Lat;

template <>
struct Lat<0> {  // D2Q9 flow + D2Q5 solute
    static constexpr int Q = 9, QS = 5, DIM = 2;
    static constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static constexpr int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    static constexpr int wn[9] = {16, 4, 4, 4, 4, 1, 1, 1, 1};
    static constexpr int SXP = 1, SXM = 3;      // solute +x / -x directions
    static constexpr int WET_SHIFT = 8;          // wet bit of solute k: WET_SHIFT + k
    static constexpr int HOP_SHIFT = 12;         // 2-hop bit of solute d: HOP_SHIFT + d
};

template <>
struct Lat<1> {  // D3Q19 flow + D3Q7 solute
    static constexpr int Q = 19, QS = 7, DIM = 3;
    static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0};
    static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 1, -1};
    static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0, -1, 1, -1, 1};
    static constexpr int opp[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
    static constexpr int wn[19] = {12, 2, 2, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
    static constexpr int SXP = 1, SXM = 2;
    static constexpr int WET_SHIFT = 18;
    static constexpr int HOP_SHIFT = 24;
};

// Link word, one uint32 per node:
//   bit i (1..Q-1)        flow: upstream node n - c_i is solid
//   bit WET_SHIFT + k     solute: link k is a wet (reactive) link of this node
//   bit HOP_SHIFT + d     solute: neighbour n + e_d is fluid and has a wet link
//                         in direction opp(d) (so this node writes its value)
//   bit 31                node is solid
constexpr uint32_t SOLID_BIT = 0x80000000u;

// ---------------------------------------------------------------------------
// Storage policies.  R = arithmetic type, T = stored type.  Each population
// is read once per pass, so the population loads are non-temporal: they
// do not displace the pseudo-potentials and indices that neighbouring
// nodes gather from the caches (measured: 0.89 -> 0.83 ms per 256^3 step).
// ---------------------------------------------------------------------------
enum { ST_F64 = 0, ST_F32 = 1, ST_F16S = 2, ST_BF16S = 3 };

template <int ST>
struct Store;

template <>
struct Store<ST_F64> {
    using R = double;
    using T = double;
    __device__ static inline R load(const T* p, R) { return __builtin_nontemporal_load(p); }
    __device__ static inline void store(T* p, R v, R) { *p = v; }
    __device__ static inline R load_plain(const T* p) { return __builtin_nontemporal_load(p); }
    __device__ static inline void store_plain(T* p, R v) { *p = v; }
};

template <>
struct Store<ST_F32> {
    using R = float;
    using T = float;
    __device__ static inline R load(const T* p, R) { return __builtin_nontemporal_load(p); }
    __device__ static inline void store(T* p, R v, R) { *p = v; }
    __device__ static inline R load_plain(const T* p) { return __builtin_nontemporal_load(p); }
    __device__ static inline void store_plain(T* p, R v) { *p = v; }
};

typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

// FP16 stores (f - shift) rounded to nearest even.
template <>
struct Store<ST_F16S> {
    using R = float;
    using T = __half;
    __device__ static inline R from_bits(uint32_t b) { return __half2float(__ushort_as_half((unsigned short)b)); }
    __device__ static inline uint32_t to_bits(R v) { return __half_as_ushort(__float2half_rn(v)); }
    // a in the low half, b in the high half, each rounded to nearest even (one packed conversion)
    __device__ static inline uint32_t pack2(R a, R b) {
        return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t){a, b}, f16x2_t));
    }
    __device__ static inline R load(const T* p, R shift) {
        return __half2float(__ushort_as_half(__builtin_nontemporal_load((const unsigned short*)p))) + shift;
    }
    __device__ static inline void store(T* p, R v, R shift) { *p = __float2half_rn(v - shift); }
    __device__ static inline R load_plain(const T* p) {
        return __half2float(__ushort_as_half(__builtin_nontemporal_load((const unsigned short*)p)));
    }
    __device__ static inline void store_plain(T* p, R v) { *p = __float2half_rn(v); }
};

// BF16: top 16 bits of the FP32 pattern, rounded to nearest even.
struct bf16_t {
    uint16_t bits;
};
__device__ __host__ static inline float bf16_to_float(uint16_t b) {
    uint32_t u = (uint32_t)b << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}
__device__ __host__ static inline uint16_t float_to_bf16_rne(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) {            // Inf / NaN: keep, quiet the NaN
        return (uint16_t)((u >> 16) | ((u & 0x007fffffu) ? 0x40u : 0u));
    }
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// On the device the conversion is the hardware one (v_cvt_pk_bf16_f32, round to
// nearest even, the same bits as float_to_bf16_rne for every non-NaN input).
__device__ static inline uint16_t bf16_rne_dev(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

template <>
struct Store<ST_BF16S> {
    using R = float;
    using T = bf16_t;
    __device__ static inline R from_bits(uint32_t b) { return bf16_to_float((uint16_t)b); }
    __device__ static inline uint32_t to_bits(R v) { return bf16_rne_dev(v); }
    __device__ static inline uint32_t pack2(R a, R b) {
        return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t){a, b}, bf16x2_t));
    }
    __device__ static inline R load(const T* p, R shift) { return bf16_to_float(__builtin_nontemporal_load(&p->bits)) + shift; }
    __device__ static inline void store(T* p, R v, R shift) { p->bits = bf16_rne_dev(v - shift); }
    __device__ static inline R load_plain(const T* p) { return bf16_to_float(__builtin_nontemporal_load(&p->bits)); }
    __device__ static inline void store_plain(T* p, R v) { p->bits = bf16_rne_dev(v); }
};

// ---------------------------------------------------------------------------
// Kernel arguments (by value).  Pointers are device pointers into the arena.
// ---------------------------------------------------------------------------
template <typename R>
struct Phys {
    int forcing;          // 0 Guo, 1 Shan-Chen velocity shift
    int solute;           // 0 off, 1 periodic, 2 inlet/outlet in x
    R inv_tau[2];         // 1 / tau_s
    R tau[2];
    R lam[2];             // 1 - 1/(2 tau_s)
    R G[2][2];
    R Gads[2];
    R rho0, inv_rho0;
    R accel[3];
    R sh[2][19];          // storage shift w_i * rhobar_s per (s, i); 0 for unshifted storage
    R Ws0, Ws;            // solute weights: rest, link
    R inv_cs2s;           // 1 / solute c_s^2
    R inv_tau_d;          // 1 / tau_d
    R wet_inv_den;        // 1 / (2 W + k tau_d / (tau_d - 1/2))
    R C_in;
    int product;          // 1: product species in solute planes QS..2QS-1
    int hplanes;          // solute planes per fluid node
    R inv_tau_d2;         // 1 / tau_d of the product
    R prod_gain;          // k tau_d2 / (tau_d2 - 1/2): product entering per unit C_b
    R C_in2;
    // per fluid node rate field (nullptr: the uniform k_wall above), two planes
    // of kstride values: 1 / (2 W + k tau_d / (tau_d - 1/2)) and k tau_d2 / (tau_d2 - 1/2)
    const R* kfield;
    unsigned kstride;
    R th_inv_tau_ef;      // 1 / tau of the fluid energy populations (conjugate heat transfer)
};

// ---------------------------------------------------------------------------
// Indexing shared by the kernel files
// ---------------------------------------------------------------------------
// element (plane j, fluid node k) of a chunked array with P planes
template <typename T>
__device__ __forceinline__ T* blk(T* base, int P, int j, unsigned k) {
    return base + ((size_t)(k >> 6) * (size_t)P + (size_t)j) * 64u + (k & 63u);
}

// Flow population arrays: plane j = s Q + i holds component s, direction i.
// With 16-bit storage and two components the two components' values of one
// direction share a 32-bit word (they are read together and pushed to the
// same node, so one load and one store move both): element (j, k) at
//   ((k >> 6) Q + i) 128 + 2 (k & 63) + s
// in stored-type units, i.e. 32-bit word ((k >> 6) Q + i) 64 + (k & 63).
// Otherwise the chunked plane layout above with P = NC Q planes.
template <int ST, int NC>
struct FlowPairs {
    static constexpr bool value = (ST >= ST_F16S) && NC == 2;
};

template <int ST, int NC, int Q>
__device__ __forceinline__ size_t fidx(int j, unsigned k) {
    if constexpr (FlowPairs<ST, NC>::value) {
        const int s = j >= Q ? 1 : 0;
        return ((size_t)(k >> 6) * Q + (size_t)(j - s * Q)) * 128u + 2u * (k & 63u) + (size_t)s;
    } else {
        return ((size_t)(k >> 6) * (size_t)(NC * Q) + (size_t)j) * 64u + (k & 63u);
    }
}

__device__ __forceinline__ void coords(const unsigned n, int nx, int ny, int& x, int& y, int& z) {
    const unsigned nxy = (unsigned)nx * (unsigned)ny;
    z = (int)(n / nxy);
    const unsigned r = n - (unsigned)z * nxy;
    y = (int)(r / (unsigned)nx);
    x = (int)(r - (unsigned)y * (unsigned)nx);
}

// box indices of the neighbourhood positions by (cx, cy, cz) in {-1,0,1}
struct NbIdx {
    unsigned xo[3];   // x - 1, x, x + 1 (wrapped)
    unsigned yo[3];   // nx * (y - 1, y, y + 1)
    unsigned zo[3];   // nx*ny * (z - 1, z, z + 1)
    __device__ __forceinline__ unsigned at(int cx, int cy, int cz) const { return xo[cx + 1] + yo[cy + 1] + zo[cz + 1]; }
};

__device__ __forceinline__ NbIdx make_nb(int x, int y, int z, int nx, int ny, int nz) {
    NbIdx b;
    b.xo[0] = x == 0 ? nx - 1 : x - 1;
    b.xo[1] = x;
    b.xo[2] = x + 1 == nx ? 0 : x + 1;
    const unsigned unx = nx, unxy = (unsigned)nx * ny;
    b.yo[0] = unx * (y == 0 ? ny - 1 : y - 1);
    b.yo[1] = unx * y;
    b.yo[2] = unx * (y + 1 == ny ? 0 : y + 1);
    b.zo[0] = unxy * (z == 0 ? nz - 1 : z - 1);
    b.zo[1] = unxy * z;
    b.zo[2] = unxy * (z + 1 == nz ? 0 : z + 1);
    return b;
}

}  // namespace mclbm
