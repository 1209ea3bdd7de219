// C ABI of the solver (declarations and contract in include/mclbm.h).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/mclbm.h"
#include "geometry.hpp"
#include "kernels.hpp"

using namespace mclbm;

namespace {

thread_local std::string g_global_error;

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int flow_q(int lat) { return lat == MCLBM_D3Q19 ? 19 : 9; }
int solute_q(int lat) { return lat == MCLBM_D3Q19 ? 7 : 5; }
size_t store_bytes(int st) { return st == MCLBM_F64 ? 8 : (st == MCLBM_F32 ? 4 : 2); }
size_t arith_bytes(int st) { return st == MCLBM_F64 ? 8 : 4; }

// ---------------------------------------------------------------- half / bf16 on the host
float half_to_float(uint16_t h) {
    const uint32_t sign = (uint32_t)(h & 0x8000u) << 16;
    uint32_t exp = (h >> 10) & 0x1fu, man = h & 0x3ffu, bits;
    if (exp == 0) {
        if (man == 0) bits = sign;
        else {  // subnormal: normalise
            int e = -1;
            do {
                man <<= 1;
                ++e;
            } while (!(man & 0x400u));
            bits = sign | ((uint32_t)(127 - 15 - e) << 23) | ((man & 0x3ffu) << 13);
        }
    } else if (exp == 31) bits = sign | 0x7f800000u | (man << 13);
    else bits = sign | ((exp + 112u) << 23) | (man << 13);
    float f;
    memcpy(&f, &bits, 4);
    return f;
}

uint16_t float_to_half_rne(float f) {
    uint32_t x;
    memcpy(&x, &f, 4);
    const uint16_t sign = (uint16_t)((x >> 16) & 0x8000u);
    const uint32_t ax = x & 0x7fffffffu;
    if (ax >= 0x7f800000u) return (uint16_t)(sign | 0x7c00u | (ax > 0x7f800000u ? 0x200u : 0u));
    if (ax >= 0x477ff000u) return (uint16_t)(sign | 0x7c00u);  // rounds to >= 65520 -> inf
    if (ax < 0x38800000u) {                                      // result subnormal or zero
        if (ax < 0x33000000u) return sign;                       // < 2^-25: rounds to 0
        const int e = (int)(ax >> 23);
        const uint32_t man = (ax & 0x7fffffu) | 0x800000u;
        const int shift = 126 - e;  // 14 - (e - 127) + 13 - 1 ... bits dropped to reach 2^-24 units
        const uint32_t q = man >> (shift - 0);
        const uint32_t rem = man & ((1u << shift) - 1u);
        const uint32_t half = 1u << (shift - 1);
        uint32_t r = q;
        if (rem > half || (rem == half && (q & 1u))) ++r;
        return (uint16_t)(sign | r);
    }
    uint32_t r = ax - 0x38000000u;  // rebias exponent (127 - 15 = 112 -> 112 << 23)
    const uint32_t rem = r & 0x1fffu;
    r >>= 13;
    if (rem > 0x1000u || (rem == 0x1000u && (r & 1u))) ++r;
    return (uint16_t)(sign | r);
}

float bf16_to_float_h(uint16_t b) {
    uint32_t u = (uint32_t)b << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}
uint16_t float_to_bf16_rne_h(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0x007fffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

}  // namespace

struct mclbm_handle {
    mclbm_params p{};
    int Q = 0, QS = 0, NC = 0;
    long long N = 0;
    hipStream_t stream = nullptr;
    void* arena = nullptr;
    bool own_arena = false;
    size_t arena_bytes = 0;
    // device regions
    void *fA = nullptr, *fB = nullptr, *hA = nullptr, *hB = nullptr;
    uint32_t* links = nullptr;
    int* map = nullptr;
    unsigned* pos = nullptr;
    void* psi = nullptr;
    void* snap = nullptr;
    double* stage = nullptr;
    double* partials = nullptr;
    double* result = nullptr;
    double* host_result = nullptr;  // pinned
    // host state
    std::vector<uint8_t> mask;
    std::vector<unsigned> pos_host;  // box index of each fluid node, increasing
    int64_t nfluid = 0;
    bool geom_set = false, fields_set = false;
    int64_t step = 0;
    bool snap_valid = false;
    double mon[16];
    double rhobar[2] = {0, 0};
    int block = 256;
    std::string err;
};

namespace {

struct Layout {
    size_t fA, fB, hA, hB, map, pos, links, psi, snap, stage, partials, result, total;
};

Ctx base_ctx(const mclbm_params& p) {
    Ctx c;
    memset(&c, 0, sizeof(c));
    c.lat = p.lattice;
    c.st = p.storage;
    c.nc = p.ncomp;
    c.nx = p.nx;
    c.ny = p.ny;
    c.nz = p.nz;
    c.N = (long long)p.nx * p.ny * p.nz;
    c.forcing = p.forcing;
    c.solute = p.solute;
    for (int s = 0; s < 2; ++s) {
        c.tau[s] = p.tau[s];
        c.Gads[s] = p.G_ads[s];
        for (int t = 0; t < 2; ++t) c.G[s][t] = p.G[s][t];
    }
    c.rho0 = p.rho0;
    for (int a = 0; a < 3; ++a) c.accel[a] = p.accel[a];
    c.D = p.D;
    c.J0 = p.J0;
    c.k_wall = p.k_wall;
    c.C_in = p.C_in;
    return c;
}

Layout layout_for(const mclbm_params& p) {
    const long long N = (long long)p.nx * p.ny * p.nz;
    const int Q = flow_q(p.lattice), QS = solute_q(p.lattice), NC = p.ncomp;
    const size_t sb = store_bytes(p.storage), ab = arith_bytes(p.storage);
    Layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = align256(off);
        off = o + bytes;
        return o;
    };
    // fluid-only arrays are sized for the worst case (every node fluid)
    const size_t M = (size_t)pad64(N);
    L.fA = take((size_t)NC * Q * M * sb);
    L.fB = take((size_t)NC * Q * M * sb);
    const size_t hb = p.solute ? (size_t)QS * M * sb : 0;
    L.hA = take(hb);
    L.hB = take(hb);
    L.map = take((size_t)N * 4);
    L.pos = take(M * 4);
    L.links = take(M * 4);
    L.psi = take((size_t)NC * N * ab);
    L.snap = take((size_t)5 * M * ab);
    L.stage = take((size_t)(NC + 4) * N * 8);
    L.partials = take(monitor_blocks_max(N) * MON_NV * 8);
    L.result = take(16 * 8);
    L.total = align256(off);
    return L;
}

bool validate(const mclbm_params* p, std::string& why) {
    char buf[256];
    if (!p) {
        why = "params is NULL";
        return false;
    }
    if (p->lattice != MCLBM_D2Q9 && p->lattice != MCLBM_D3Q19) {
        why = "unknown lattice";
        return false;
    }
    if (p->nx < 1 || p->ny < 1 || p->nz < 1 || p->ny > 65535 || p->nz > 65535) {
        why = "dimensions must be >= 1 (ny, nz <= 65535)";
        return false;
    }
    if (p->lattice == MCLBM_D2Q9 && p->nz != 1) {
        why = "D2Q9 needs nz == 1";
        return false;
    }
    if ((long long)p->nx * p->ny * p->nz >= (1LL << 31)) {
        why = "lattice has more than 2^31 - 1 nodes";
        return false;
    }
    if (p->ncomp != 1 && p->ncomp != 2) {
        why = "ncomp must be 1 or 2";
        return false;
    }
    if (p->forcing != MCLBM_FORCING_GUO && p->forcing != MCLBM_FORCING_SC) {
        why = "unknown forcing scheme";
        return false;
    }
    if (p->solute < MCLBM_SOLUTE_OFF || p->solute > MCLBM_SOLUTE_INLET_OUTLET_X) {
        why = "unknown solute mode";
        return false;
    }
    if (p->solute == MCLBM_SOLUTE_INLET_OUTLET_X && p->nx < 2) {
        why = "inlet/outlet solute needs nx >= 2";
        return false;
    }
    if (p->storage < MCLBM_F64 || p->storage > MCLBM_BF16_SHIFT) {
        why = "unknown storage";
        return false;
    }
    if (p->monitor_every < 1) {
        why = "monitor_every must be >= 1";
        return false;
    }
    if (p->reserved != 0) {
        why = "reserved field must be 0";
        return false;
    }
    for (int s = 0; s < p->ncomp; ++s)
        if (!(p->tau[s] > 0.5) || !isfinite(p->tau[s])) {
            snprintf(buf, sizeof buf, "tau[%d] = %g must be > 1/2", s, p->tau[s]);
            why = buf;
            return false;
        }
    if (!(p->rho0 > 0) || !isfinite(p->rho0)) {
        why = "rho0 must be > 0";
        return false;
    }
    if (p->solute) {
        if (!(p->D > 0) || !isfinite(p->D)) {
            why = "solute diffusivity D must be > 0";
            return false;
        }
        if (!(p->J0 >= 0 && p->J0 < 1)) {
            why = "J0 must be in [0, 1)";
            return false;
        }
        if (!(p->k_wall >= 0) || !isfinite(p->k_wall)) {
            why = "k_wall must be >= 0";
            return false;
        }
    }
    return true;
}

int fail(mclbm_handle* h, int code, const std::string& msg) {
    if (h) h->err = msg;
    else g_global_error = msg;
    return code;
}

int hip_fail(mclbm_handle* h, hipError_t e, const char* what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(h, MCLBM_EHIP, m);
}

#define HIPCHK(h, expr)                                     \
    do {                                                    \
        hipError_t e_ = (expr);                             \
        if (e_ != hipSuccess) return hip_fail(h, e_, #expr); \
    } while (0)

Ctx make_ctx(mclbm_handle* h) {
    Ctx c = base_ctx(h->p);
    c.rhobar[0] = h->rhobar[0];
    c.rhobar[1] = h->rhobar[1];
    c.stream = h->stream;
    c.fA = h->fA;
    c.fB = h->fB;
    c.hA = h->hA;
    c.hB = h->hB;
    c.Nf = h->nfluid;
    c.links = h->links;
    c.pos = h->pos;
    c.map = h->map;
    c.psi = h->psi;
    c.snap = h->snap;
    c.partials = h->partials;
    c.result = h->result;
    c.block = h->block;
    return c;
}

double ratio(double num, double den) {
    if (den == 0.0) return num == 0.0 ? 0.0 : INFINITY;
    return sqrt(num / den);
}

// read the monitor result into h->mon; returns 1 if it counted non-finite values
int collect_monitor(mclbm_handle* h, bool had_snapshot) {
    const double* r = h->host_result;
    for (int k = 0; k < 16; ++k) h->mon[k] = 0.0;
    h->mon[0] = (double)h->step;
    h->mon[1] = r[0];
    h->mon[2] = h->NC == 2 ? r[1] : 0.0;
    h->mon[3] = r[2];
    if (had_snapshot) {
        h->mon[4] = ratio(r[3], r[4]);
        h->mon[5] = ratio(r[5], r[6]);
        h->mon[6] = ratio(r[7], r[8]);
    } else {
        h->mon[4] = h->mon[5] = h->mon[6] = INFINITY;
        if (h->NC == 1) h->mon[5] = 0.0;
        if (!h->p.solute) h->mon[6] = 0.0;
    }
    if (h->NC == 1) h->mon[5] = 0.0;
    if (!h->p.solute) h->mon[6] = 0.0;
    h->mon[7] = r[9];
    h->mon[8] = r[10];
    h->mon[9] = std::max(h->mon[4], std::max(h->mon[5], h->mon[6]));
    h->mon[10] = (double)h->step;
    return r[9] != 0.0 || !isfinite(r[0]) || !isfinite(r[2]);
}

int run_monitor(mclbm_handle* h) {
    Ctx c = make_ctx(h);
    const bool had = h->snap_valid;
    HIPCHK(h, k_monitor(c, had ? 1 : 0));
    HIPCHK(h, hipMemcpyAsync(h->host_result, h->result, 16 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    h->snap_valid = true;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (collect_monitor(h, had)) return fail(h, MCLBM_EDIVERGED, "non-finite value at a monitor");
    return MCLBM_OK;
}

}  // namespace

extern "C" {

int mclbm_required_bytes(const mclbm_params* p, size_t* bytes) {
    std::string why;
    if (!validate(p, why)) return fail(nullptr, MCLBM_EINVAL, why);
    if (!bytes) return fail(nullptr, MCLBM_EINVAL, "bytes is NULL");
    *bytes = layout_for(*p).total;
    return MCLBM_OK;
}

int mclbm_init_lattice(const mclbm_params* p, void* device_arena, size_t arena_bytes, void* hip_stream,
                       mclbm_handle** out) {
    std::string why;
    if (!out) return fail(nullptr, MCLBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!validate(p, why)) return fail(nullptr, MCLBM_EINVAL, why);
    Layout L = layout_for(*p);
    if (device_arena && arena_bytes < L.total) {
        char buf[160];
        snprintf(buf, sizeof buf, "arena of %zu bytes is smaller than the %zu bytes required", arena_bytes, L.total);
        return fail(nullptr, MCLBM_ENOMEM, buf);
    }
    if (device_arena && ((uintptr_t)device_arena & 255u))
        return fail(nullptr, MCLBM_EINVAL, "arena must be 256-byte aligned");
    mclbm_handle* h = new mclbm_handle();
    h->p = *p;
    h->Q = flow_q(p->lattice);
    h->QS = solute_q(p->lattice);
    h->NC = p->ncomp;
    h->N = (long long)p->nx * p->ny * p->nz;
    h->stream = (hipStream_t)hip_stream;
    for (int k = 0; k < 16; ++k) h->mon[k] = 0.0;
    h->mon[0] = -1.0;
    if (device_arena) {
        h->arena = device_arena;
        h->arena_bytes = arena_bytes;
    } else {
        hipError_t e = hipMalloc(&h->arena, L.total);
        if (e != hipSuccess) {
            delete h;
            return fail(nullptr, MCLBM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        h->own_arena = true;
        h->arena_bytes = L.total;
    }
    char* base = (char*)h->arena;
    h->fA = base + L.fA;
    h->fB = base + L.fB;
    h->hA = p->solute ? base + L.hA : nullptr;
    h->hB = p->solute ? base + L.hB : nullptr;
    h->links = (uint32_t*)(base + L.links);
    h->map = (int*)(base + L.map);
    h->pos = (unsigned*)(base + L.pos);
    h->psi = base + L.psi;
    h->snap = base + L.snap;
    h->stage = (double*)(base + L.stage);
    h->partials = (double*)(base + L.partials);
    h->result = (double*)(base + L.result);
    hipError_t e = hipHostMalloc((void**)&h->host_result, 16 * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) {
        if (h->own_arena) (void)hipFree(h->arena);
        delete h;
        return fail(nullptr, MCLBM_EHIP, std::string("hipHostMalloc: ") + hipGetErrorString(e));
    }
    *out = h;
    return MCLBM_OK;
}

int mclbm_set_geometry(mclbm_handle* h, const uint8_t* solid_mask, int64_t* n_reclassified) {
    if (!h) return MCLBM_EINVAL;
    if (!solid_mask) return fail(h, MCLBM_EINVAL, "solid_mask is NULL");
    h->mask.assign(solid_mask, solid_mask + h->N);
    for (auto& m : h->mask) m = m ? 1 : 0;
    GeomSpec gs{h->p.lattice, h->p.nx, h->p.ny, h->p.nz, h->p.solute};
    const int64_t nrc = pinch_fill(gs, h->mask);
    int64_t nf = 0;
    for (auto m : h->mask) nf += (m == 0);
    if (n_reclassified) *n_reclassified = nrc;
    if (nf == 0) {
        h->geom_set = false;
        return fail(h, MCLBM_EINVAL, "no fluid node left after reclassification");
    }
    std::vector<uint32_t> words;
    link_words(gs, h->mask, words, nullptr, nullptr);
    // fluid numbering in increasing box index; link words of fluid nodes only
    const long long N = h->N;
    h->pos_host.clear();
    h->pos_host.reserve((size_t)nf);
    std::vector<int> map((size_t)N, -1);
    for (long long n = 0; n < N; ++n)
        if (!h->mask[n]) {
            map[n] = (int)h->pos_host.size();
            h->pos_host.push_back((unsigned)n);
        }
    std::vector<uint32_t> fw((size_t)nf);
    for (int64_t k = 0; k < nf; ++k) fw[k] = words[h->pos_host[k]];
    HIPCHK(h, hipMemcpyAsync(h->map, map.data(), (size_t)N * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->pos, h->pos_host.data(), (size_t)nf * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->links, fw.data(), (size_t)nf * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->nfluid = nf;
    h->geom_set = true;
    h->fields_set = false;
    return MCLBM_OK;
}

int mclbm_get_geometry(mclbm_handle* h, uint8_t* mask_out, uint32_t* flow_links, uint32_t* solute_links) {
    if (!h) return MCLBM_EINVAL;
    if (!h->geom_set) return fail(h, MCLBM_ESTATE, "set_geometry has not been called");
    if (mask_out) memcpy(mask_out, h->mask.data(), (size_t)h->N);
    if (flow_links || solute_links) {
        std::vector<uint32_t> words, fb, sb;
        GeomSpec gs{h->p.lattice, h->p.nx, h->p.ny, h->p.nz, h->p.solute};
        link_words(gs, h->mask, words, &fb, &sb);
        if (flow_links) memcpy(flow_links, fb.data(), (size_t)h->N * 4);
        if (solute_links) memcpy(solute_links, sb.data(), (size_t)h->N * 4);
    }
    return MCLBM_OK;
}

int mclbm_init_fields(mclbm_handle* h, const double* rho, const double* u, const double* C) {
    if (!h) return MCLBM_EINVAL;
    if (!h->geom_set) return fail(h, MCLBM_ESTATE, "set_geometry has not been called");
    if (!rho) return fail(h, MCLBM_EINVAL, "rho is NULL");
    const long long N = h->N;
    for (int s = 0; s < h->NC; ++s) {
        double sum = 0.0;
        for (long long n = 0; n < N; ++n) {
            if (h->mask[n]) continue;
            const double r = rho[s * N + n];
            if (!(r > 0.0) || !isfinite(r)) return fail(h, MCLBM_EINVAL, "rho must be > 0 and finite on fluid nodes");
            sum += r;
        }
        h->rhobar[s] = sum / (double)h->nfluid;
    }
    double* st_rho = h->stage;
    double* st_u = h->stage + (size_t)h->NC * N;
    double* st_C = h->stage + (size_t)(h->NC + 3) * N;
    HIPCHK(h, hipMemcpyAsync(st_rho, rho, (size_t)h->NC * N * 8, hipMemcpyHostToDevice, h->stream));
    if (u) HIPCHK(h, hipMemcpyAsync(st_u, u, (size_t)3 * N * 8, hipMemcpyHostToDevice, h->stream));
    if (C && h->p.solute) HIPCHK(h, hipMemcpyAsync(st_C, C, (size_t)N * 8, hipMemcpyHostToDevice, h->stream));
    Ctx c = make_ctx(h);
    HIPCHK(h, k_init(c, st_rho, u ? st_u : nullptr, (C && h->p.solute) ? st_C : nullptr));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->step = 0;
    h->snap_valid = false;
    for (int k = 0; k < 16; ++k) h->mon[k] = 0.0;
    h->mon[0] = -1.0;
    h->fields_set = true;
    return MCLBM_OK;
}

int mclbm_step(mclbm_handle* h, int64_t n) {
    if (!h) return MCLBM_EINVAL;
    if (n < 0) return fail(h, MCLBM_EINVAL, "n must be >= 0");
    if (!h->fields_set) return fail(h, MCLBM_ESTATE, "init_fields has not been called");
    const int K = h->p.monitor_every;
    bool monitored = false, had = false;
    for (int64_t s = 0; s < n; ++s) {
        Ctx c = make_ctx(h);
        HIPCHK(h, k_step(c));
        std::swap(h->fA, h->fB);
        std::swap(h->hA, h->hB);
        ++h->step;
        if (h->step % K == 0) {
            Ctx cm = make_ctx(h);
            had = h->snap_valid;
            HIPCHK(h, k_monitor(cm, had ? 1 : 0));
            h->snap_valid = true;
            monitored = true;
        }
    }
    if (monitored) {
        HIPCHK(h, hipMemcpyAsync(h->host_result, h->result, 16 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        if (collect_monitor(h, had)) return fail(h, MCLBM_EDIVERGED, "non-finite value at a monitor");
    }
    return MCLBM_OK;
}

int mclbm_monitor_now(mclbm_handle* h) {
    if (!h) return MCLBM_EINVAL;
    if (!h->fields_set) return fail(h, MCLBM_ESTATE, "init_fields has not been called");
    return run_monitor(h);
}

int mclbm_get_moments(mclbm_handle* h, double* rho, double* u, double* C, int32_t dst_is_device) {
    if (!h) return MCLBM_EINVAL;
    if (!h->fields_set) return fail(h, MCLBM_ESTATE, "init_fields has not been called");
    Ctx c = make_ctx(h);
    const long long N = h->N;
    if (dst_is_device) {
        HIPCHK(h, k_moments(c, rho, u, C));
        return MCLBM_OK;
    }
    double* st_rho = h->stage;
    double* st_u = h->stage + (size_t)h->NC * N;
    double* st_C = h->stage + (size_t)(h->NC + 3) * N;
    HIPCHK(h, k_moments(c, rho ? st_rho : nullptr, u ? st_u : nullptr, C ? st_C : nullptr));
    if (rho) HIPCHK(h, hipMemcpyAsync(rho, st_rho, (size_t)h->NC * N * 8, hipMemcpyDeviceToHost, h->stream));
    if (u) HIPCHK(h, hipMemcpyAsync(u, st_u, (size_t)3 * N * 8, hipMemcpyDeviceToHost, h->stream));
    if (C) HIPCHK(h, hipMemcpyAsync(C, st_C, (size_t)N * 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return MCLBM_OK;
}

int mclbm_get_monitors(mclbm_handle* h, double out[16]) {
    if (!h || !out) return MCLBM_EINVAL;
    for (int k = 0; k < 16; ++k) out[k] = h->mon[k];
    out[10] = (double)h->step;
    return MCLBM_OK;
}

int mclbm_population_bytes(mclbm_handle* h, int32_t raw, size_t* bytes) {
    if (!h || !bytes) return MCLBM_EINVAL;
    const size_t nval = (size_t)(h->NC * h->Q + (h->p.solute ? h->QS : 0)) * (size_t)h->N;
    *bytes = nval * (raw ? store_bytes(h->p.storage) : 8);
    return MCLBM_OK;
}

// Position of (plane j, fluid node k) in a blocked fluid-only array with P planes.
static inline size_t blk_index(size_t P, size_t j, size_t k) { return ((k >> 6) * P + j) * 64 + (k & 63); }

int mclbm_get_populations(mclbm_handle* h, void* dst, int32_t raw) {
    if (!h || !dst) return MCLBM_EINVAL;
    if (!h->fields_set) return fail(h, MCLBM_ESTATE, "init_fields has not been called");
    const size_t sb = store_bytes(h->p.storage);
    const size_t M = (size_t)pad64(h->nfluid);
    const size_t PF = (size_t)h->NC * h->Q, PS = h->p.solute ? (size_t)h->QS : 0;
    std::vector<unsigned char> dev((PF + PS) * M * sb);
    HIPCHK(h, hipMemcpyAsync(dev.data(), h->fA, PF * M * sb, hipMemcpyDeviceToHost, h->stream));
    if (PS) HIPCHK(h, hipMemcpyAsync(dev.data() + PF * M * sb, h->hA, PS * M * sb, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    const size_t N = (size_t)h->N;
    const Ctx c = make_ctx(h);
    const size_t nplanes = PF + PS;
    if (raw) {
        unsigned char* out = (unsigned char*)dst;
        memset(out, 0, nplanes * N * sb);
        for (size_t j = 0; j < nplanes; ++j) {
            const bool flow = j < PF;
            const unsigned char* src = flow ? dev.data() : dev.data() + PF * M * sb;
            const size_t P = flow ? PF : PS, jj = flow ? j : j - PF;
            for (size_t k = 0; k < (size_t)h->nfluid; ++k)
                memcpy(out + (j * N + h->pos_host[k]) * sb, src + blk_index(P, jj, k) * sb, sb);
        }
        return MCLBM_OK;
    }
    double* out = (double*)dst;
    memset(out, 0, nplanes * N * sizeof(double));
    for (size_t j = 0; j < nplanes; ++j) {
        const bool flow = j < PF;
        const unsigned char* src = flow ? dev.data() : dev.data() + PF * M * sb;
        const size_t P = flow ? PF : PS, jj = flow ? j : j - PF;
        const int s = flow ? (int)(j / h->Q) : 0, i = flow ? (int)(j % h->Q) : 0;
        const float shift = flow ? shift_f32(c, s, i) : 0.0f;
        for (size_t k = 0; k < (size_t)h->nfluid; ++k) {
            const size_t q = blk_index(P, jj, k);
            double v;
            switch (h->p.storage) {
                case MCLBM_F64: v = ((const double*)src)[q]; break;
                case MCLBM_F32: v = ((const float*)src)[q]; break;
                case MCLBM_F16_SHIFT: v = (double)(half_to_float(((const uint16_t*)src)[q]) + shift); break;
                default: v = (double)(bf16_to_float_h(((const uint16_t*)src)[q]) + shift); break;
            }
            out[j * N + h->pos_host[k]] = v;
        }
    }
    return MCLBM_OK;
}

int mclbm_set_populations(mclbm_handle* h, const void* src, int32_t raw) {
    if (!h || !src) return MCLBM_EINVAL;
    if (!h->fields_set) return fail(h, MCLBM_ESTATE, "init_fields has not been called");
    const size_t sb = store_bytes(h->p.storage);
    const size_t M = (size_t)pad64(h->nfluid);
    const size_t PF = (size_t)h->NC * h->Q, PS = h->p.solute ? (size_t)h->QS : 0;
    const size_t N = (size_t)h->N, nplanes = PF + PS;
    std::vector<unsigned char> dev((PF + PS) * M * sb, 0);
    const Ctx c = make_ctx(h);
    for (size_t j = 0; j < nplanes; ++j) {
        const bool flow = j < PF;
        unsigned char* dstp = flow ? dev.data() : dev.data() + PF * M * sb;
        const size_t P = flow ? PF : PS, jj = flow ? j : j - PF;
        const int s = flow ? (int)(j / h->Q) : 0, i = flow ? (int)(j % h->Q) : 0;
        const float shift = flow ? shift_f32(c, s, i) : 0.0f;
        for (size_t k = 0; k < (size_t)h->nfluid; ++k) {
            const size_t q = blk_index(P, jj, k), n = h->pos_host[k];
            if (raw) {
                memcpy(dstp + q * sb, (const unsigned char*)src + (j * N + n) * sb, sb);
                continue;
            }
            const double v = ((const double*)src)[j * N + n];
            switch (h->p.storage) {
                case MCLBM_F64: ((double*)dstp)[q] = v; break;
                case MCLBM_F32: ((float*)dstp)[q] = (float)v; break;
                case MCLBM_F16_SHIFT: ((uint16_t*)dstp)[q] = float_to_half_rne((float)v - shift); break;
                default: ((uint16_t*)dstp)[q] = float_to_bf16_rne_h((float)v - shift); break;
            }
        }
    }
    HIPCHK(h, hipMemcpyAsync(h->fA, dev.data(), PF * M * sb, hipMemcpyHostToDevice, h->stream));
    if (PS) HIPCHK(h, hipMemcpyAsync(h->hA, dev.data() + PF * M * sb, PS * M * sb, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return MCLBM_OK;
}

int mclbm_run_to_residual(mclbm_handle* h, double tol, int64_t max_steps, int64_t* steps_taken) {
    if (!h) return MCLBM_EINVAL;
    if (!h->fields_set) return fail(h, MCLBM_ESTATE, "init_fields has not been called");
    if (max_steps < 0) return fail(h, MCLBM_EINVAL, "max_steps must be >= 0");
    const int K = h->p.monitor_every;
    int64_t taken = 0;
    int rc = 1;
    while (taken < max_steps) {
        int64_t chunk = K - (h->step % K);
        if (chunk > max_steps - taken) chunk = max_steps - taken;
        const int64_t before = h->step;
        int e = mclbm_step(h, chunk);
        taken += h->step - before;
        if (e != MCLBM_OK) {
            if (steps_taken) *steps_taken = taken;
            return e;
        }
        if (h->step % K == 0 && h->mon[0] == (double)h->step && h->mon[9] <= tol) {
            rc = MCLBM_OK;
            break;
        }
    }
    if (steps_taken) *steps_taken = taken;
    return rc;
}

int mclbm_set_launch(mclbm_handle* h, int32_t block_threads) {
    if (!h) return MCLBM_EINVAL;
    if (block_threads != 64 && block_threads != 128 && block_threads != 256)
        return fail(h, MCLBM_EINVAL, "block_threads must be 64, 128 or 256");
    h->block = block_threads;
    return MCLBM_OK;
}

int mclbm_get_step(mclbm_handle* h, int64_t* step) {
    if (!h || !step) return MCLBM_EINVAL;
    *step = h->step;
    return MCLBM_OK;
}

int mclbm_synchronize(mclbm_handle* h) {
    if (!h) return MCLBM_EINVAL;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return MCLBM_OK;
}

void mclbm_destroy(mclbm_handle* h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    if (h->host_result) (void)hipHostFree(h->host_result);
    if (h->own_arena && h->arena) (void)hipFree(h->arena);
    delete h;
}

const char* mclbm_last_error(const mclbm_handle* h) {
    if (!h) return g_global_error.c_str();
    return h->err.c_str();
}

}  // extern "C"
