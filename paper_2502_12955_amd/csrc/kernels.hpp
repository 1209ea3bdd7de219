// Host-side interface of the kernel file: type-erased launch context.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "common.hpp"

namespace mclbm {

// Geometry of one sample of a batch (a single lattice is a batch of one).
struct SampleDev {
    int nx, ny, nz;   // box dimensions
    int Nf;           // fluid nodes
    int N;            // box nodes
    int dbase;        // first box node of the sample in the concatenated dense arrays
    int kbase;        // first fluid index of the sample (multiple of 64)
    int pad_;
};

struct Ctx {
    int lat, st, nc;            // lattice (0 D2Q9, 1 D3Q19), storage, components
    int nsamples;
    long long Ntot;             // box nodes of all samples
    long long max_sample_nodes; // box nodes of the largest sample
    long long nchunks;          // 64-node chunks of the fluid numbering (with per-sample padding)
    int forcing, solute;
    double tau[2], G[2][2], Gads[2], rho0, accel[3];
    double D, J0, k_wall, C_in;
    const void* kfield;         // per fluid node reaction rate (arith type) or nullptr: k_wall
    int product;                // second solute species produced at the reacting walls
    int hplanes;                // solute planes per fluid node (QS per species, 0 without solute)
    double D2, C_in2;
    double rhobar[2];           // storage shift (used by *_SHIFT storage only)
    hipStream_t stream;
    void *fA, *fB, *hA, *hB;    // populations (current state in A), blocks of 64 fluid nodes
    const SampleDev* smp;       // [nsamples]
    const int* chunk_sample;    // [nchunks] sample owning each 64-node chunk
    const unsigned* pos;        // [nchunks*64] box index (within its sample) of fluid node k
    const int* map;             // [Ntot] fluid index of box node, -1 if solid
    const uint32_t* links;      // [nchunks*64] link words
    void* psi;                  // pseudo-potentials [nchunks*64][nc] in the fluid numbering (arith type)
    void* snap;                 // residual snapshot [5][nchunks*64] (arith type)
    const int* work;            // active chunk list (device) or nullptr = every chunk
    const int* nwork;           // device count of `work`
    long long nactive;          // host copy of that count (grid sizes)
    double* partials;           // [nchunks][MON_NV] per-chunk monitor partials
    double* result;             // [nsamples][16] per-sample monitor sums
    int block;                  // threads per block of the step kernels (64, 128, 256)
    int grid;                   // persistent grid (blocks, multiple of 8); 0 = one pass over the chunks
    int flat;                   // 1: flat 64-bit addresses in the collide pass even where buffer offsets fit
    // conjugate heat transfer (single lattice; 0 = off)
    int thermal;
    double th_tau_ef, th_tau_es, th_rhocp_f, th_rhocp_s, th_h_r, th_A, th_EoR, th_tol;
    int th_maxit;
    void *gA, *gB;              // fluid energy populations, fluid chunks, Q planes
    void *gsA, *gsB;            // solid energy populations, solid-list chunks, Q planes
    void* Ti;                   // [niface] interface temperatures (arith type)
    const int* smap;            // [N] solid-list index of a box node, -1 for a pure fluid node
    const unsigned* spos;       // [nsolid] box index of each solid-list node
    long long nsolid;           // solid and interface nodes
    const int* iface;           // [niface][4]: fluid index, solid-list index, unknown-solid bits, 0
    long long niface;
    int thermal_nx, thermal_ny, thermal_nz;   // the lattice (thermal runs are single lattices)
    long long thermal_nfluid;               // fluid nodes
    unsigned long long* th_stats;   // [2] device counters: iterations, unsettled solves
};

constexpr int MON_NV = 11;      // values reduced per monitor

inline long long pad64(long long n) { return (n + 63) & ~63LL; }
// Population-shift value of component s, direction i, exactly as the kernels use it.
float shift_f32(const Ctx& c, int s, int i);

// Kernel-argument block for arithmetic type R (float or double).
template <typename R>
Phys<R> make_phys(const Ctx& c);

hipError_t k_init(const Ctx& c, const double* rho, const double* u, const double* C);
hipError_t k_step(const Ctx& c);
// conjugate heat transfer: the solid energy pass and the interface solve of a
// step (after the collide pass, before the A/B swap); initial energy populations
// from FP64 box fields T [N] and u [3][N] (u may be NULL); one output plane in
// FP64 box layout (what 0: temperature, 1: fluid energy plane i, 2: solid energy
// plane i; nodes without that field get 0)
hipError_t k_thermal_step(const Ctx& c);
hipError_t k_thermal_init(const Ctx& c, const double* T, const double* u);
hipError_t k_thermal_out(const Ctx& c, int what, int plane, double* dst);
hipError_t k_moments(const Ctx& c, double* rho, double* u, double* C);
hipError_t k_monitor(const Ctx& c, int have_snapshot);
// FP64 values src[0 .. cnt-1] stored into elements q0 .. q0 + cnt - 1 of the
// chunked array dst of `planes` planes with the step kernels' encoder (flow = 1:
// a flow array with per-plane storage shifts; 0: unshifted solute planes)
hipError_t k_encode_planes(const Ctx& c, const double* src, void* dst, long long q0, long long cnt, int planes,
                          int flow);
// particle deposition after a step: dep[k] += DP * C at fluid nodes with a solid
// neighbour; *count (zeroed by the caller) receives the nodes whose deposit exceeds 1
hipError_t k_deposit_step(const Ctx& c, double* dep, double DP, int* count);
// renumbering after a geometry change: dst(j, k) = src(j, from[k]) over planes of
// elem_bytes-wide values in the chunked layout, 0 where from[k] < 0 (remap.hip)
hipError_t k_remap_planes(void* dst, const void* src, int planes, const int* from, long long nnew, int elem_bytes,
                          hipStream_t stream);

}  // namespace mclbm
