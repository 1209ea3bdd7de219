// Fused single-pass step: one kernel per time step.
//
// The force at a node needs the pseudo-potential of its neighbours at the
// same time level, i.e. the densities of nodes one link away, whose
// populations belong to other threads.  Instead of a separate density sweep
// (an extra read of every population), each workgroup owns a 64 x TY tile of
// an (x, y) plane and marches along z through a chunk of planes:
//
//   for plane z:  load populations of plane z+1 (tile + one-node halo ring),
//                 compute rho and psi of plane z+1 into an LDS ring slot,
//                 barrier,
//                 collide plane z (populations held in registers since the
//                 previous iteration, neighbour psi from LDS planes z-1, z, z+1),
//                 push-stream into buffer B.
//
// Interior populations are read from HBM once per step; only the halo ring
// and the two extra planes per z-chunk are re-read (mostly cache hits).  A
// 4-slot LDS ring needs one barrier per plane: the slot written for z+2 is
// the one last read while colliding z-2.  Workgroups are remapped so that
// consecutive tiles land on the same XCD (round-robin dispatch over 8 XCDs),
// which keeps the halo rows of neighbouring tiles in the same L2.
//
// Addressing: a wavefront is one x-row of the tile, so the row (and every
// neighbour row) is wave-uniform.  Every access is a wave-uniform plane base
// (scalar registers) plus a 32-bit node offset, which the loads and stores
// take directly; the plane loop costs no vector address arithmetic.  The z
// loop is unrolled by two with two register sets (no copies between planes).
#include "common.hpp"
#include "kernels.hpp"
#include "node.hpp"

namespace mclbm {

constexpr int FTX = 64;  // tile width along x: one wavefront per row

template <int LAT, int ST, int NC, int TY>
__global__ void __launch_bounds__(FTX * TY) k_fused(Phys<typename Store<ST>::R> P, int N,
                                                    const typename Store<ST>::T* __restrict__ fA,
                                                    typename Store<ST>::T* __restrict__ fB,
                                                    const typename Store<ST>::T* __restrict__ hA,
                                                    typename Store<ST>::T* __restrict__ hB,
                                                    const uint32_t* __restrict__ links, int ntx, int nty,
                                                    int zchunk, int nblocks, int per_xcd) {
    using L = Lat<LAT>;
    using S = Store<ST>;
    using R = typename S::R;
    using T = typename S::T;
    constexpr int Q = L::Q, QS = L::QS;
    constexpr int NT = FTX * TY;
    constexpr int LW = FTX + 2, LH = TY + 2, PLANE = LW * LH;
    constexpr int H = 2 * LW + 2 * TY;              // halo nodes per plane
    constexpr int HPT = (H + NT - 1) / NT;          // halo nodes per thread (max)
    extern __shared__ unsigned char smem_raw[];
    R* lds = reinterpret_cast<R*>(smem_raw);        // [4][NC][LH][LW]

    // XCD-aware tile order: block b runs on XCD b % 8; give each XCD a
    // contiguous range of tiles.
    const int b = blockIdx.x;
    const int tile = (b & 7) * per_xcd + (b >> 3);
    if (tile >= nblocks) return;
    const int tx = tile % ntx;
    const int rest = tile / ntx;
    const int ty = rest % nty;
    const int zc = rest / nty;
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const int x0 = tx * FTX, y0 = ty * TY;
    const int z0 = (LAT == 1) ? zc * zchunk : 0;
    const int z1 = (LAT == 1) ? min(z0 + zchunk, nz) : 1;

    const int t = threadIdx.x;
    const int lane = t & (FTX - 1);
    const int ly = __builtin_amdgcn_readfirstlane(t / FTX);  // wave-uniform row of the tile
    const unsigned gx = (unsigned)((x0 + lane) % nx);
    const int gy = (y0 + ly) % ny;
    const bool valid = (x0 + lane < nx) && (y0 + ly < ny);
    const unsigned xm = gx == 0 ? nx - 1 : gx - 1, xp = gx + 1 == (unsigned)nx ? 0 : gx + 1;
    const int ym = gy == 0 ? ny - 1 : gy - 1, yp = gy + 1 == ny ? 0 : gy + 1;
    const int nxy = nx * ny;

    // halo assignment: LDS position and in-plane node offset (wrapped)
    int hpos[HPT];
    unsigned hoff[HPT];
#pragma unroll
    for (int k = 0; k < HPT; ++k) {
        const int hh = t + k * NT;
        int jx = 0, jy = 0;
        if (hh < LW) {
            jx = hh;
            jy = 0;
        } else if (hh < 2 * LW) {
            jx = hh - LW;
            jy = LH - 1;
        } else if (hh < 2 * LW + TY) {
            jx = 0;
            jy = hh - 2 * LW + 1;
        } else {
            jx = LW - 1;
            jy = hh - 2 * LW - TY + 1;
        }
        const int hx = ((x0 - 1 + jx) % nx + nx) % nx;
        const int hy = ((y0 - 1 + jy) % ny + ny) % ny;
        hpos[k] = (hh < H) ? jy * LW + jx : -1;
        hoff[k] = (unsigned)(hx + nx * hy);
    }

    R sh[NC][Q];
    load_shifts<LAT, ST, NC>(P, sh);

    // plane j of an SoA array, addressed with a 32-bit byte offset (fits: N * sizeof(T) < 2^32)
    auto ld = [&](const T* base, int j, unsigned boff, R shift) -> R {
        const T* p = reinterpret_cast<const T*>(reinterpret_cast<const char*>(base + (size_t)j * (size_t)N) + boff);
        return S::load(p, shift);
    };
    auto ldp = [&](const T* base, int j, unsigned boff) -> R {
        const T* p = reinterpret_cast<const T*>(reinterpret_cast<const char*>(base + (size_t)j * (size_t)N) + boff);
        return S::load_plain(p);
    };
    auto st = [&](T* base, int j, unsigned boff, R v, R shift) {
        T* p = reinterpret_cast<T*>(reinterpret_cast<char*>(base + (size_t)j * (size_t)N) + boff);
        S::store(p, v, shift);
    };
    auto stp = [&](T* base, int j, unsigned boff, R v) {
        T* p = reinterpret_cast<T*>(reinterpret_cast<char*>(base + (size_t)j * (size_t)N) + boff);
        S::store_plain(p, v);
    };
    constexpr unsigned TB = sizeof(T);

    auto psi_of = [&](const R (&ff)[NC][Q], int s) -> R {
        R r = 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) r += ff[s][i];
        return P.rho0 * (R(1) - exp_r<R>(-r * P.inv_rho0));
    };

    // Load plane zz into (fo, ho, lwo) for the interior node; halo psi; psi -> LDS slot.
    auto load_plane = [&](int zz, int slot, R (&fo)[NC][Q], R (&ho)[QS], uint32_t& lwo) {
        const unsigned zoff = (unsigned)(nxy * zz);
        const unsigned n = gx + (unsigned)(nx * gy) + zoff;
        const unsigned nb_ = n * TB;
        lwo = links[n];
        R* sl = lds + slot * NC * PLANE;
        if (!(lwo & SOLID_BIT)) {
#pragma unroll
            for (int s = 0; s < NC; ++s)
#pragma unroll
                for (int i = 0; i < Q; ++i) fo[s][i] = ld(fA, s * Q + i, nb_, sh[s][i]);
            if (P.solute && valid) {
#pragma unroll
                for (int k = 0; k < QS; ++k) ho[k] = ldp(hA, k, nb_);
            }
#pragma unroll
            for (int s = 0; s < NC; ++s) sl[s * PLANE + (ly + 1) * LW + (lane + 1)] = psi_of(fo, s);
        } else {
#pragma unroll
            for (int s = 0; s < NC; ++s) sl[s * PLANE + (ly + 1) * LW + (lane + 1)] = R(0);
        }
#pragma unroll
        for (int k = 0; k < HPT; ++k) {
            if (hpos[k] < 0) continue;
            const unsigned m = hoff[k] + zoff;
            const unsigned mb = m * TB;
            const uint32_t lh = links[m];
            R ps[NC];
#pragma unroll
            for (int s = 0; s < NC; ++s) ps[s] = R(0);
            if (!(lh & SOLID_BIT)) {
                R fh[NC][Q];
#pragma unroll
                for (int s = 0; s < NC; ++s)
#pragma unroll
                    for (int i = 0; i < Q; ++i) fh[s][i] = ld(fA, s * Q + i, mb, sh[s][i]);
#pragma unroll
                for (int s = 0; s < NC; ++s) ps[s] = psi_of(fh, s);
            }
#pragma unroll
            for (int s = 0; s < NC; ++s) sl[s * PLANE + hpos[k]] = ps[s];
        }
    };

    // Collide the held plane z (populations fo) and push into B.
    auto collide_plane = [&](int z, R (&fo)[NC][Q], R (&ho)[QS], uint32_t lwo) {
        const int s_prev = (z - z0) & 3, s_cur = (z - z0 + 1) & 3, s_next = (z - z0 + 2) & 3;
        if (!(valid && !(lwo & SOLID_BIT))) return;
        const R* lp = lds + s_prev * NC * PLANE;
        const R* lc = lds + s_cur * NC * PLANE;
        const R* ln = lds + s_next * NC * PLANE;
        auto nb = [&](int tc, int i) -> R {
            const R* base = (L::cz[i] < 0) ? lp : ((L::cz[i] > 0) ? ln : lc);
            return base[tc * PLANE + (ly + 1 + L::cy[i]) * LW + (lane + 1 + L::cx[i])];
        };
        R u[3];
        flow_collide<LAT, NC, R>(P, lwo, fo, nb, u);

        // wave-uniform neighbour-row offsets
        const int zm = (LAT == 1) ? (z == 0 ? nz - 1 : z - 1) : z;
        const int zp = (LAT == 1) ? (z + 1 == nz ? 0 : z + 1) : z;
        auto rowoff = [&](int cy, int cz) -> unsigned {
            const int yy = cy < 0 ? ym : (cy > 0 ? yp : gy);
            const int zz = cz < 0 ? zm : (cz > 0 ? zp : z);
            return (unsigned)(nx * yy + nxy * zz);
        };
        const unsigned own = (gx + rowoff(0, 0)) * TB;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const unsigned xd = L::cx[i] < 0 ? xm : (L::cx[i] > 0 ? xp : gx);
            const unsigned dst = (xd + rowoff(L::cy[i], L::cz[i])) * TB;
            const bool bb = (i != 0) && (lwo & (1u << L::opp[i]));
#pragma unroll
            for (int s = 0; s < NC; ++s) {
                if (bb) st(fB, s * Q + L::opp[i], own, fo[s][i], sh[s][i]);
                else st(fB, s * Q + i, dst, fo[s][i], sh[s][i]);
            }
        }
        if (P.solute) {
            solute_collide<LAT, R>(P, ho, u);
            stp(hB, 0, own, ho[0]);
            const bool seam_mode = (P.solute == 2);
#pragma unroll
            for (int d = 1; d < QS; ++d) {
                const int dx = L::cx[d];
                const bool seam = seam_mode && ((gx + 1 == (unsigned)nx && dx == 1) || (gx == 0 && dx == -1));
                if (!seam && !(lwo & (1u << L::opp[d]))) {
                    const unsigned xd = dx < 0 ? xm : (dx > 0 ? xp : gx);
                    const unsigned dst = (xd + rowoff(L::cy[d], L::cz[d])) * TB;
                    stp(hB, d, dst, ho[d]);
                    if (lwo & (1u << (L::HOP_SHIFT + d))) {
                        const R Cb = R(2) * ho[d] * P.wet_inv_den;
                        stp(hB, L::opp[d], dst, R(2) * P.Ws * Cb - ho[d]);
                    }
                    if (seam_mode && d == L::SXM && gx == 1)
                        stp(hB, L::SXP, dst, R(2) * P.Ws * P.C_in - ho[d]);
                }
                if (seam_mode && d == L::SXM && gx + 1 == (unsigned)nx) stp(hB, d, own, ho[d]);
            }
        }
    };

    R fa[NC][Q], fb[NC][Q];
    R ha[QS], hb[QS];
    uint32_t lwa, lwb;
#pragma unroll
    for (int k = 0; k < QS; ++k) ha[k] = hb[k] = R(0);
    if (LAT == 1) load_plane(z0 == 0 ? nz - 1 : z0 - 1, 0, fb, hb, lwb);
    load_plane(z0, 1, fa, ha, lwa);

    if (LAT == 0) {
        __syncthreads();
        collide_plane(0, fa, ha, lwa);
        return;
    }
    for (int z = z0; z < z1; z += 2) {
        load_plane(z + 1 == nz ? 0 : z + 1, (z - z0 + 2) & 3, fb, hb, lwb);
        __syncthreads();
        collide_plane(z, fa, ha, lwa);
        if (z + 1 >= z1) break;
        load_plane(z + 2 >= nz ? z + 2 - nz : z + 2, (z - z0 + 3) & 3, fa, ha, lwa);
        __syncthreads();
        collide_plane(z + 1, fb, hb, lwb);
    }
}

template <int LAT, int ST, int NC, int TY>
static hipError_t launch_fused(const Ctx& c) {
    using R = typename Store<ST>::R;
    using T = typename Store<ST>::T;
    auto P = make_phys<R>(c);
    const int ntx = (c.nx + FTX - 1) / FTX;
    const int nty = (c.ny + TY - 1) / TY;
    const int zchunk = (LAT == 1) ? (c.zchunk > 0 ? c.zchunk : c.nz) : 1;
    const int nzc = (LAT == 1) ? (c.nz + zchunk - 1) / zchunk : 1;
    const long long nb = (long long)ntx * nty * nzc;
    if (nb >= (1LL << 31) / 8) return hipErrorInvalidConfiguration;
    const int per_xcd = (int)((nb + 7) / 8);
    const size_t lds = (size_t)4 * NC * (FTX + 2) * (TY + 2) * sizeof(R);
    if (lds > 65536) return hipErrorInvalidConfiguration;
    if ((unsigned long long)c.N * sizeof(T) >= (1ULL << 32)) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((k_fused<LAT, ST, NC, TY>), dim3(8 * per_xcd), dim3(FTX * TY), lds, c.stream, P, (int)c.N,
                       (const T*)c.fA, (T*)c.fB, (const T*)c.hA, (T*)c.hB, c.links, ntx, nty, zchunk, (int)nb,
                       per_xcd);
    return hipGetLastError();
}

template <int LAT, int ST, int NC>
hipError_t step_fused(const Ctx& c) {
    switch (c.tile_y) {
        case 1: return launch_fused<LAT, ST, NC, 1>(c);
        case 2: return launch_fused<LAT, ST, NC, 2>(c);
        case 4: return launch_fused<LAT, ST, NC, 4>(c);
        case 8: return launch_fused<LAT, ST, NC, 8>(c);
        case 16: return launch_fused<LAT, ST, NC, 16>(c);
        default: return hipErrorInvalidValue;
    }
}

#define INST(L, S, C) template hipError_t step_fused<L, S, C>(const Ctx&);
INST(0, 0, 1) INST(0, 0, 2) INST(0, 1, 1) INST(0, 1, 2) INST(0, 2, 1) INST(0, 2, 2) INST(0, 3, 1) INST(0, 3, 2)
INST(1, 0, 1) INST(1, 0, 2) INST(1, 1, 1) INST(1, 1, 2) INST(1, 2, 1) INST(1, 2, 2) INST(1, 3, 1) INST(1, 3, 2)

}  // namespace mclbm
