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
    long long N;
    int forcing, solute;
    double tau[2], G[2][2], Gads[2], rho0, accel[3];
    double D, J0, k_wall, C_in;
    double rhobar[2];           // storage shift (used by *_SHIFT storage only)
    hipStream_t stream;
    void *fA, *fB, *hA, *hB;    // populations (current state in A)
    const uint32_t* links;      // link words
    void* psi;                  // pseudo-potential field [nc][N] (arith type)
    void* snap;                 // residual snapshot [5][N] (arith type)
    double* partials;           // monitor block partials
    double* result;             // monitor result [16]
    int variant;                // 0 fused, 1 two-pass
    int tile_x, tile_y, zchunk; // fused-kernel tile
};

constexpr int MON_NV = 11;      // values reduced per monitor

// Number of monitor blocks (partials rows) for this lattice.
size_t monitor_blocks(const Ctx& c);
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
