// Host-side interface of the kernel file: type-erased launch context.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "common.hpp"

namespace mclbm {

struct Ctx {
    int lat, st, nc;            // lattice (0 D2Q9, 1 D3Q19), storage, components
    int nx, ny, nz;
    long long N;                // box nodes
    long long Nf;               // fluid nodes
    int forcing, solute;
    double tau[2], G[2][2], Gads[2], rho0, accel[3];
    double D, J0, k_wall, C_in;
    double rhobar[2];           // storage shift (used by *_SHIFT storage only)
    hipStream_t stream;
    void *fA, *fB, *hA, *hB;    // populations (current state in A)
    const unsigned* pos;        // [Nf] box index of fluid node k
    const int* map;             // [N] fluid index of box node n, -1 if solid
    const uint32_t* links;      // [Nf] link words
    void* psi;                  // pseudo-potential field [nc][N] (arith type, 0 on solids)
    void* snap;                 // residual snapshot [5][Nf] (arith type)
    double* partials;           // monitor block partials
    double* result;             // monitor result [16]
    int block;                  // threads per block of the step kernels (64..256)
};

constexpr int MON_NV = 11;      // values reduced per monitor

// Number of monitor blocks (partials rows) for this lattice, and its bound for N nodes.
size_t monitor_blocks(const Ctx& c);
size_t monitor_blocks_max(long long N);
// Padded fluid count: populations are stored in blocks of 64 nodes.
inline long long pad64(long long n) { return (n + 63) & ~63LL; }
// Population-shift value of component s, direction i, exactly as the kernels use it.
float shift_f32(const Ctx& c, int s, int i);

// Kernel-argument block for arithmetic type R (float or double).
template <typename R>
Phys<R> make_phys(const Ctx& c);

hipError_t k_init(const Ctx& c, const double* rho, const double* u, const double* C);
hipError_t k_step(const Ctx& c);
hipError_t k_moments(const Ctx& c, double* rho, double* u, double* C);
hipError_t k_monitor(const Ctx& c, int have_snapshot);

}  // namespace mclbm
