// C ABI of the solver (declarations and contract in include/mclbm.h).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cstdio>
#include <string>
#include <vector>

#include "mclbm.h"
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

float bf16_to_float_h(uint16_t b) {
    uint32_t u = (uint32_t)b << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

}  // namespace

struct SampleHost {
    int nx, ny, nz;
    long long N;      // box nodes
    long long dbase;  // first box node in the concatenated dense arrays
    long long kbase;  // first fluid index (multiple of 64)
    long long nf;     // fluid nodes
    std::vector<uint8_t> mask;
    std::vector<unsigned> pos;  // box index of each fluid node, in the fluid numbering (band order)
    std::vector<uint32_t> words;  // link word of each fluid node (kept for deposition runs)
    bool frozen = false;        // converged or diverged, excluded from the work list
    long long conv_step = -1;
    long long div_step = -1;    // monitor step at which a non-finite value was seen
    bool bad = false;           // the last monitor saw a non-finite value
    double mon[16];
};

struct mclbm_handle {
    mclbm_params p{};  // physics (sample 0's dimensions)
    int Q = 0, QS = 0, NC = 0;
    int HP = 0;        // solute planes per fluid node: QS per species, 0 without solute
    int S = 0;
    std::vector<SampleHost> smp;
    long long Ntot = 0;      // box nodes of all samples
    long long Mmax = 0;      // fluid-node capacity (sum of padded box sizes)
    long long nchunks = 0;   // chunks of the current fluid numbering
    hipStream_t stream = nullptr;
    void* arena = nullptr;
    bool own_arena = false;
    size_t arena_bytes = 0;
    // device regions
    void *fA = nullptr, *fB = nullptr, *hA = nullptr, *hB = nullptr;
    void* kfield = nullptr;   // per fluid node reaction rate (arithmetic type), rate_field only
    double* dep = nullptr;    // per fluid node particle deposit C_ps, deposition only
    int* dep_count = nullptr; // per step of a batch: deposits above 1 after that step
    void* dep_snap = nullptr; // populations (A) and deposits at the start of a batch
    uint32_t* links = nullptr;
    int* map = nullptr;
    unsigned* pos = nullptr;
    void* psi = nullptr;
    void* snap = nullptr;
    double* stage = nullptr;
    double* partials = nullptr;
    double* result = nullptr;
    SampleDev* smp_dev = nullptr;
    int* chunk_sample = nullptr;
    int* work = nullptr;
    int* nwork = nullptr;
    long long nactive = 0;          // chunks in the work list
    double* host_result = nullptr;  // pinned [S][16]
    int* host_nwork = nullptr;      // pinned
    int* host_dep = nullptr;        // pinned [DEP_BATCH], deposition only
    int64_t dep_converted = 0;      // nodes turned solid by deposition since init_fields
    int dep_batch = 64;             // steps of the next speculative deposition batch
    std::vector<double> k_box;      // the caller's rate field, re-applied after a deposition rebuild
    // state
    bool geom_set = false, fields_set = false;
    int64_t step = 0;
    bool snap_valid = false;
    double mon[16];
    double rhobar[2] = {0, 0};
    int block = 256, grid = 0;
    int bands = 0;                  // y-bands of the fluid numbering (0: eight, one per XCD)
    int flat = 0;                   // 1: flat 64-bit addressing in the collide pass
    // conjugate heat transfer (library-owned device memory, allocated in set_geometry)
    bool thermal = false, temp_set = false;
    mclbm_thermal th{};
    void *gA = nullptr, *gB = nullptr, *gsA = nullptr, *gsB = nullptr, *Ti = nullptr;
    int* smap = nullptr;
    unsigned* spos = nullptr;
    int* iface = nullptr;
    unsigned long long* th_stats = nullptr;
    long long nsolid = 0, niface = 0, ndegenerate = 0;
    // graph replay of monitor_every steps (one per A/B parity)
    bool use_graph = false;
    hipStream_t gstream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    std::string err;
};

namespace {

// steps per speculative batch of a deposition run (one synchronisation each)
constexpr int DEP_BATCH = 64;

struct Layout {
    size_t fA, fB, hA, hB, kfield, dep, depcnt, dsnap, map, pos, links, psi, snap, stage, partials, result, smp, chunk_sample,
        work, nwork, total;
};

Ctx base_ctx(const mclbm_params& p) {
    Ctx c;
    memset(&c, 0, sizeof(c));
    c.lat = p.lattice;
    c.st = p.storage;
    c.nc = p.ncomp;
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
    c.product = p.solute ? p.product : 0;
    c.D2 = p.D2;
    c.C_in2 = p.C_in2;
    c.hplanes = p.solute ? solute_q(p.lattice) * (1 + c.product) : 0;
    c.kfield = nullptr;
    return c;
}

Layout layout_for(const mclbm_params* ps, int n) {
    const mclbm_params& p = ps[0];
    const int Q = flow_q(p.lattice), QS = solute_q(p.lattice), NC = p.ncomp;
    const size_t sb = store_bytes(p.storage), ab = arith_bytes(p.storage);
    long long Ntot = 0, M = 0;
    for (int s = 0; s < n; ++s) {
        const long long N = (long long)ps[s].nx * ps[s].ny * ps[s].nz;
        Ntot += N;
        M += pad64(N);  // capacity: every node fluid
    }
    const size_t nch = (size_t)(M / 64);
    Layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = align256(off);
        off = o + bytes;
        return o;
    };
    L.fA = take((size_t)NC * Q * M * sb);
    L.fB = take((size_t)NC * Q * M * sb);
    const size_t hb = p.solute ? (size_t)QS * (p.product ? 2 : 1) * M * sb : 0;
    L.hA = take(hb);
    L.hB = take(hb);
    L.kfield = take(p.solute && p.rate_field ? (size_t)2 * M * ab : 0);
    L.dep = take(p.deposition ? (size_t)M * 8 : 0);
    L.depcnt = take(p.deposition ? DEP_BATCH * 4 : 0);
    L.dsnap = take(p.deposition ? (size_t)NC * Q * M * sb + hb + (size_t)M * 8 : 0);
    L.map = take((size_t)Ntot * 4);
    L.pos = take((size_t)M * 4);
    L.links = take((size_t)M * 4);
    L.psi = take((size_t)NC * M * ab);
    L.snap = take((size_t)5 * M * ab);
    L.stage = take((size_t)(NC + 4 + (p.solute && p.product ? 1 : 0)) * Ntot * 8);
    L.partials = take(nch * MON_NV * 8);
    L.result = take((size_t)n * 16 * 8);
    L.smp = take((size_t)n * sizeof(SampleDev));
    L.chunk_sample = take(nch * 4);
    L.work = take(nch * 4);
    L.nwork = take(64);
    L.total = align256(off);
    return L;
}

bool validate_one(const mclbm_params* p, std::string& why) {
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
    if (p->reserved != 0 || p->reserved2 != 0) {
        why = "reserved fields must be 0";
        return false;
    }
    if ((p->deposition != 0 && p->deposition != 1) || (p->deposition && !p->solute)) {
        why = "deposition must be 0 or 1, and 1 needs the solute on";
        return false;
    }
    if (p->deposition && (!(p->dep_prob > 0) || !isfinite(p->dep_prob))) {
        why = "deposition probability dep_prob must be > 0";
        return false;
    }
    if ((p->rate_field != 0 && p->rate_field != 1) || (p->rate_field && !p->solute)) {
        why = "rate_field must be 0 or 1, and 1 needs the solute on";
        return false;
    }
    if (p->product != 0 && p->product != 1) {
        why = "product must be 0 or 1";
        return false;
    }
    if (p->product && !p->solute) {
        why = "the product species needs the solute on";
        return false;
    }
    if (p->product && (!(p->D2 > 0) || !isfinite(p->D2))) {
        why = "product diffusivity D2 must be > 0";
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

// every sample valid, same physics as sample 0, sizes within the 32-bit indexing
bool validate(const mclbm_params* p, int n, std::string& why) {
    if (!p || n < 1) {
        why = "need at least one sample";
        return false;
    }
    if (n > 1 && p[0].deposition) {
        why = "deposition needs a single lattice (a batch of one)";
        return false;
    }
    long long Ntot = 0, M = 0;
    for (int s = 0; s < n; ++s) {
        if (!validate_one(&p[s], why)) {
            if (n > 1) why = "sample " + std::to_string(s) + ": " + why;
            return false;
        }
        mclbm_params a = p[0], b = p[s];
        a.nx = b.nx;
        a.ny = b.ny;
        a.nz = b.nz;
        if (memcmp(&a, &b, sizeof(a)) != 0) {
            why = "sample " + std::to_string(s) + " differs from sample 0 in more than its dimensions";
            return false;
        }
        const long long N = (long long)p[s].nx * p[s].ny * p[s].nz;
        Ntot += N;
        M += pad64(N);
    }
    const int Q = flow_q(p[0].lattice);
    if (M * (long long)(p[0].ncomp * Q) >= (1LL << 32) || Ntot >= (1LL << 31)) {
        why = "lattice too large for 32-bit node indexing";
        return false;
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

#define HIPCHK(h, expr)                                      \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return hip_fail(h, e_, #expr); \
    } while (0)

Ctx make_ctx(mclbm_handle* h, hipStream_t stream) {
    Ctx c = base_ctx(h->p);
    c.nsamples = h->S;
    c.Ntot = h->Ntot;
    c.flat = h->flat;
    c.thermal = h->thermal && h->gA ? 1 : 0;
    if (c.thermal) {
        c.th_tau_ef = h->th.tau_ef;
        c.th_tau_es = h->th.tau_es;
        c.th_rhocp_f = h->th.rhocp_f;
        c.th_rhocp_s = h->th.rhocp_s;
        c.th_h_r = h->th.h_r;
        c.th_A = h->th.A;
        c.th_EoR = h->th.E_over_R;
        c.th_tol = h->th.T_tol;
        c.th_maxit = h->th.T_maxit;
        c.gA = h->gA;
        c.gB = h->gB;
        c.gsA = h->gsA;
        c.gsB = h->gsB;
        c.Ti = h->Ti;
        c.smap = h->smap;
        c.spos = h->spos;
        c.nsolid = h->nsolid;
        c.iface = h->iface;
        c.niface = h->niface;
        c.th_stats = h->th_stats;
        c.thermal_nx = h->smp[0].nx;
        c.thermal_ny = h->smp[0].ny;
        c.thermal_nz = h->smp[0].nz;
        c.thermal_nfluid = h->smp[0].nf;
    }
    c.max_sample_nodes = 0;
    for (const auto& sm : h->smp) c.max_sample_nodes = std::max(c.max_sample_nodes, sm.N);
    c.nchunks = h->nchunks;
    c.rhobar[0] = h->rhobar[0];
    c.rhobar[1] = h->rhobar[1];
    c.stream = stream;
    c.fA = h->fA;
    c.fB = h->fB;
    c.hA = h->hA;
    c.hB = h->hB;
    c.kfield = h->kfield;
    c.smp = h->smp_dev;
    c.chunk_sample = h->chunk_sample;
    c.pos = h->pos;
    c.map = h->map;
    c.links = h->links;
    c.psi = h->psi;
    c.snap = h->snap;
    // the work list only once some sample has converged: with every sample
    // running, chunk = item saves a dependent load at the start of each chunk
    bool any_frozen = false;
    for (const auto& sm : h->smp) any_frozen |= sm.frozen;
    c.work = any_frozen ? h->work : nullptr;
    c.nwork = h->nwork;
    c.nactive = h->nactive;
    c.partials = h->partials;
    c.result = h->result;
    c.block = h->block;
    c.grid = h->grid;
    return c;
}
Ctx make_ctx(mclbm_handle* h) { return make_ctx(h, h->stream); }

double ratio(double num, double den) {
    if (den == 0.0) return num == 0.0 ? 0.0 : INFINITY;
    return sqrt(num / den);
}

void drop_graphs(mclbm_handle* h) {
    for (auto& g : h->gexec)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
}

// Monitor values of one sample from the raw sums r[0..10].
void sample_monitor(mclbm_handle* h, SampleHost& sm, const double* r, bool had) {
    double* m = sm.mon;
    for (int k = 0; k < 16; ++k) m[k] = 0.0;
    m[0] = (double)h->step;
    m[1] = r[0];
    m[2] = h->NC == 2 ? r[1] : 0.0;
    m[3] = r[2];
    m[4] = had ? ratio(r[3], r[4]) : INFINITY;
    m[5] = (h->NC == 1) ? 0.0 : (had ? ratio(r[5], r[6]) : INFINITY);
    m[6] = (!h->p.solute) ? 0.0 : (had ? ratio(r[7], r[8]) : INFINITY);
    m[7] = r[9];
    m[8] = r[10];
    m[9] = std::max(m[4], std::max(m[5], m[6]));
    m[10] = (double)h->step;
    m[11] = (double)sm.conv_step;
    m[12] = sm.frozen ? 1.0 : 0.0;
}

// Aggregate over samples: masses and counts summed, residuals the maximum over
// the samples still running (all samples if none is frozen).
void aggregate_monitor(mclbm_handle* h) {
    double* m = h->mon;
    for (int k = 0; k < 16; ++k) m[k] = 0.0;
    m[0] = h->smp[0].mon[0];
    bool any_active = false;
    for (auto& s : h->smp) any_active |= !s.frozen;
    for (auto& s : h->smp) {
        for (int k : {1, 2, 3, 7, 8}) m[k] += s.mon[k];
        if (!any_active || !s.frozen)
            for (int k : {4, 5, 6, 9}) m[k] = std::max(m[k], s.mon[k]);
    }
    m[10] = (double)h->step;
}

// Read the monitor results of the last monitor launch (stream already ordered).
int collect_monitor(mclbm_handle* h, bool had) {
    HIPCHK(h, hipMemcpyAsync(h->host_result, h->result, (size_t)h->S * 16 * sizeof(double), hipMemcpyDeviceToHost,
                             h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    bool bad = false;
    for (int s = 0; s < h->S; ++s) {
        SampleHost& sm = h->smp[s];
        if (sm.frozen) continue;
        const double* r = h->host_result + (size_t)s * 16;
        sample_monitor(h, sm, r, had);
        sm.bad = r[9] != 0.0 || !isfinite(r[0]) || !isfinite(r[2]);
        bad |= sm.bad;
    }
    aggregate_monitor(h);
    if (bad) return fail(h, MCLBM_EDIVERGED, "non-finite value at a monitor");
    return MCLBM_OK;
}

// Upload the list of chunks of the samples that are not frozen.
int upload_work(mclbm_handle* h) {
    std::vector<int> w;
    w.reserve((size_t)h->nchunks);
    for (auto& s : h->smp) {
        if (s.frozen) continue;
        const long long c0 = s.kbase / 64, nc = (s.nf + 63) / 64;
        for (long long c = 0; c < nc; ++c) w.push_back((int)(c0 + c));
    }
    *h->host_nwork = (int)w.size();
    h->nactive = (long long)w.size();
    if (!w.empty())
        HIPCHK(h, hipMemcpyAsync(h->work, w.data(), w.size() * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->nwork, h->host_nwork, 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return MCLBM_OK;
}

// Position of (plane j, fluid node k) in a chunked fluid-only array with P planes.
static inline size_t blk_index(size_t P, size_t j, size_t k) { return ((k >> 6) * P + j) * 64 + (k & 63); }
// flow arrays with 16-bit storage of two components pair the components of a
// direction in one 32-bit word (the device-side fidx): element (j, k) at
// ((k >> 6) Q + i) 128 + 2 (k & 63) + s with j = s Q + i
static inline bool flow_pairs(const mclbm_handle* h) {
    return (h->p.storage == MCLBM_F16_SHIFT || h->p.storage == MCLBM_BF16_SHIFT) && h->NC == 2;
}
static inline size_t flow_index(const mclbm_handle* h, size_t j, size_t k) {
    const size_t Q = (size_t)h->Q;
    if (flow_pairs(h)) {
        const size_t s = j >= Q ? 1 : 0;
        return ((k >> 6) * Q + (j - s * Q)) * 128 + 2 * (k & 63) + s;
    }
    return blk_index((size_t)h->NC * Q, j, k);
}

// Copy a frozen sample's current state into buffer B as well, so that later
// A/B swaps keep presenting its final state.
int mirror_sample(mclbm_handle* h, const SampleHost& s) {
    const size_t sb = store_bytes(h->p.storage);
    const size_t PF = (size_t)h->NC * h->Q, PS = (size_t)h->HP;
    const size_t c0 = (size_t)(s.kbase / 64), nc = (size_t)((s.nf + 63) / 64);
    HIPCHK(h, hipMemcpyAsync((char*)h->fB + c0 * PF * 64 * sb, (char*)h->fA + c0 * PF * 64 * sb, nc * PF * 64 * sb,
                             hipMemcpyDeviceToDevice, h->stream));
    if (PS)
        HIPCHK(h, hipMemcpyAsync((char*)h->hB + c0 * PS * 64 * sb, (char*)h->hA + c0 * PS * 64 * sb,
                                 nc * PS * 64 * sb, hipMemcpyDeviceToDevice, h->stream));
    return MCLBM_OK;
}

// Launch one step (density + collide) on `stream` and swap A/B.
int launch_step(mclbm_handle* h, hipStream_t stream) {
    Ctx c = make_ctx(h, stream);
    HIPCHK(h, k_step(c));
    std::swap(h->fA, h->fB);
    std::swap(h->hA, h->hB);
    std::swap(h->gA, h->gB);
    std::swap(h->gsA, h->gsB);
    ++h->step;
    return MCLBM_OK;
}

// Capture monitor_every steps plus the monitor into a graph for the current
// A/B parity (requires an even monitor_every so that the parity returns).
int graph_for_parity(mclbm_handle* h, int parity, hipGraphExec_t* out) {
    if (h->gexec[parity]) {
        *out = h->gexec[parity];
        return MCLBM_OK;
    }
    if (!h->gstream) {
        HIPCHK(h, hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking));
        HIPCHK(h, hipEventCreateWithFlags(&h->ev_in, hipEventDisableTiming));
        HIPCHK(h, hipEventCreateWithFlags(&h->ev_out, hipEventDisableTiming));
    }
    const int K = h->p.monitor_every;
    const int64_t step0 = h->step;
    void *fA = h->fA, *fB = h->fB, *hA = h->hA, *hB = h->hB;
    void *gA = h->gA, *gB = h->gB, *gsA = h->gsA, *gsB = h->gsB;
    HIPCHK(h, hipStreamBeginCapture(h->gstream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int s = 0; s < K && e == hipSuccess; ++s) {
        Ctx c = make_ctx(h, h->gstream);
        e = k_step(c);
        std::swap(h->fA, h->fB);
        std::swap(h->hA, h->hB);
        std::swap(h->gA, h->gB);
        std::swap(h->gsA, h->gsB);
    }
    if (e == hipSuccess) e = k_monitor(make_ctx(h, h->gstream), 1);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(h->gstream, &graph);
    h->fA = fA, h->fB = fB, h->hA = hA, h->hB = hB;
    h->gA = gA, h->gB = gB, h->gsA = gsA, h->gsB = gsB;
    h->step = step0;
    if (e != hipSuccess) return hip_fail(h, e, "capture");
    if (e2 != hipSuccess) return hip_fail(h, e2, "hipStreamEndCapture");
    hipError_t e3 = hipGraphInstantiate(&h->gexec[parity], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) return hip_fail(h, e3, "hipGraphInstantiate");
    *out = h->gexec[parity];
    return MCLBM_OK;
}

// Run one full monitor interval through the graph (caller checks alignment).
int replay_interval(mclbm_handle* h) {
    // which of the two arena buffers currently holds the state selects the graph
    const int p = h->fA < h->fB ? 0 : 1;
    hipGraphExec_t ge = nullptr;
    int rc = graph_for_parity(h, p, &ge);
    if (rc != MCLBM_OK) return rc;
    HIPCHK(h, hipEventRecord(h->ev_in, h->stream));
    HIPCHK(h, hipStreamWaitEvent(h->gstream, h->ev_in, 0));
    HIPCHK(h, hipGraphLaunch(ge, h->gstream));
    HIPCHK(h, hipEventRecord(h->ev_out, h->gstream));
    HIPCHK(h, hipStreamWaitEvent(h->stream, h->ev_out, 0));
    h->step += h->p.monitor_every;  // K even: A/B assignment unchanged
    return MCLBM_OK;
}

}  // namespace

extern "C" {

int mclbm_required_bytes_batch(const mclbm_params* p, int32_t n, size_t* bytes) {
    std::string why;
    if (!validate(p, n, why)) return fail(nullptr, MCLBM_EINVAL, why);
    if (!bytes) return fail(nullptr, MCLBM_EINVAL, "bytes is NULL");
    *bytes = layout_for(p, n).total;
    return MCLBM_OK;
}

int mclbm_required_bytes(const mclbm_params* p, size_t* bytes) { return mclbm_required_bytes_batch(p, 1, bytes); }

int mclbm_init_batch(const mclbm_params* p, int32_t n, void* device_arena, size_t arena_bytes, void* hip_stream,
                     mclbm_handle** out) {
    std::string why;
    if (!out) return fail(nullptr, MCLBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!validate(p, n, why)) return fail(nullptr, MCLBM_EINVAL, why);
    Layout L = layout_for(p, n);
    if (device_arena && arena_bytes < L.total) {
        char buf[160];
        snprintf(buf, sizeof buf, "arena of %zu bytes is smaller than the %zu bytes required", arena_bytes, L.total);
        return fail(nullptr, MCLBM_ENOMEM, buf);
    }
    if (device_arena && ((uintptr_t)device_arena & 255u))
        return fail(nullptr, MCLBM_EINVAL, "arena must be 256-byte aligned");
    mclbm_handle* h = new mclbm_handle();
    h->p = p[0];
    h->Q = flow_q(p[0].lattice);
    h->QS = solute_q(p[0].lattice);
    h->HP = p[0].solute ? h->QS * (p[0].product ? 2 : 1) : 0;
    h->NC = p[0].ncomp;
    h->S = n;
    h->smp.resize(n);
    long long dbase = 0;
    for (int s = 0; s < n; ++s) {
        SampleHost& sm = h->smp[s];
        sm.nx = p[s].nx;
        sm.ny = p[s].ny;
        sm.nz = p[s].nz;
        sm.N = (long long)sm.nx * sm.ny * sm.nz;
        sm.dbase = dbase;
        sm.kbase = 0;
        sm.nf = 0;
        for (int k = 0; k < 16; ++k) sm.mon[k] = 0.0;
        sm.mon[0] = -1.0;
        dbase += sm.N;
        h->Mmax += pad64(sm.N);
    }
    h->Ntot = dbase;
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
    h->hA = p[0].solute ? base + L.hA : nullptr;
    h->hB = p[0].solute ? base + L.hB : nullptr;
    h->kfield = (p[0].solute && p[0].rate_field) ? base + L.kfield : nullptr;
    h->dep = p[0].deposition ? (double*)(base + L.dep) : nullptr;
    h->dep_count = p[0].deposition ? (int*)(base + L.depcnt) : nullptr;
    h->dep_snap = p[0].deposition ? base + L.dsnap : nullptr;
    h->map = (int*)(base + L.map);
    h->pos = (unsigned*)(base + L.pos);
    h->links = (uint32_t*)(base + L.links);
    h->psi = base + L.psi;
    h->snap = base + L.snap;
    h->stage = (double*)(base + L.stage);
    h->partials = (double*)(base + L.partials);
    h->result = (double*)(base + L.result);
    h->smp_dev = (SampleDev*)(base + L.smp);
    h->chunk_sample = (int*)(base + L.chunk_sample);
    h->work = (int*)(base + L.work);
    h->nwork = (int*)(base + L.nwork);
    hipError_t e = hipHostMalloc((void**)&h->host_result, (size_t)n * 16 * sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&h->host_nwork, 64, hipHostMallocDefault);
    if (e == hipSuccess && p[0].deposition) e = hipHostMalloc((void**)&h->host_dep, DEP_BATCH * 4, hipHostMallocDefault);
    if (e != hipSuccess) {
        if (h->host_result) (void)hipHostFree(h->host_result);
        if (h->host_nwork) (void)hipHostFree(h->host_nwork);
        if (h->own_arena) (void)hipFree(h->arena);
        delete h;
        return fail(nullptr, MCLBM_EHIP, std::string("hipHostMalloc: ") + hipGetErrorString(e));
    }
    *out = h;
    return MCLBM_OK;
}

int mclbm_init_lattice(const mclbm_params* p, void* device_arena, size_t arena_bytes, void* hip_stream,
                       mclbm_handle** out) {
    return mclbm_init_batch(p, 1, device_arena, arena_bytes, hip_stream, out);
}

// ---------------------------------------------------------------- conjugate heat transfer
static void free_thermal(mclbm_handle* h) {
    for (void** p : {&h->gA, &h->gB, &h->gsA, &h->gsB, &h->Ti, (void**)&h->smap, (void**)&h->spos,
                     (void**)&h->iface, (void**)&h->th_stats})
        if (*p) {
            (void)hipFree(*p);
            *p = nullptr;
        }
    h->nsolid = h->niface = h->ndegenerate = 0;
    h->temp_set = false;
}

static int band_rows(int ny, int bands);

// Build the solid list, the interface list and the thermal arrays for the
// current geometry (single lattice).  `map` is the box -> fluid index map.
static int build_thermal(mclbm_handle* h, const std::vector<int>& map) {
    free_thermal(h);
    SampleHost& sm = h->smp[0];
    const GeomSpec gs{h->p.lattice, sm.nx, sm.ny, sm.nz, h->p.solute};
    std::vector<unsigned> spos, ibox;
    std::vector<int> smap;
    std::vector<uint32_t> msb;
    thermal_lists(gs, sm.mask, band_rows(sm.ny, h->bands), spos, smap, ibox, msb);
    const int Q = h->Q;
    const size_t sb = store_bytes(h->p.storage), ab = arith_bytes(h->p.storage);
    const long long nsol = (long long)spos.size(), ni = (long long)ibox.size();
    const long long schunks = std::max(1LL, pad64(nsol) / 64);
    std::vector<int> iface((size_t)std::max(1LL, ni) * 4, 0);
    for (long long q = 0; q < ni; ++q) {
        const unsigned n = ibox[(size_t)q];
        iface[(size_t)(4 * q)] = map[n];
        iface[(size_t)(4 * q + 1)] = smap[n];
        iface[(size_t)(4 * q + 2)] = (int)msb[(size_t)q];
    }
    const size_t gbytes = (size_t)h->nchunks * 64 * Q * sb, gsbytes = (size_t)schunks * 64 * Q * sb;
    auto dalloc = [&](void** p, size_t bytes) -> hipError_t { return hipMalloc(p, std::max(bytes, (size_t)256)); };
    hipError_t e = dalloc(&h->gA, gbytes);
    if (e == hipSuccess) e = dalloc(&h->gB, gbytes);
    if (e == hipSuccess) e = dalloc(&h->gsA, gsbytes);
    if (e == hipSuccess) e = dalloc(&h->gsB, gsbytes);
    if (e == hipSuccess) e = dalloc(&h->Ti, (size_t)std::max(1LL, ni) * ab);
    if (e == hipSuccess) e = dalloc((void**)&h->smap, smap.size() * 4);
    if (e == hipSuccess) e = dalloc((void**)&h->spos, (size_t)schunks * 64 * 4);
    if (e == hipSuccess) e = dalloc((void**)&h->iface, iface.size() * 4);
    if (e == hipSuccess) e = dalloc((void**)&h->th_stats, 64);
    if (e != hipSuccess) {
        free_thermal(h);
        return fail(h, MCLBM_ENOMEM, std::string("thermal arrays: ") + hipGetErrorString(e));
    }
    spos.resize((size_t)schunks * 64, 0u);
    HIPCHK(h, hipMemcpyAsync(h->smap, smap.data(), smap.size() * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->spos, spos.data(), spos.size() * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->iface, iface.data(), iface.size() * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemsetAsync(h->th_stats, 0, 64, h->stream));
    // the energy arrays hold no stale values in slots the kernels never write
    HIPCHK(h, hipMemsetAsync(h->gA, 0, gbytes, h->stream));
    HIPCHK(h, hipMemsetAsync(h->gB, 0, gbytes, h->stream));
    HIPCHK(h, hipMemsetAsync(h->gsA, 0, gsbytes, h->stream));
    HIPCHK(h, hipMemsetAsync(h->gsB, 0, gsbytes, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    // degenerate interface nodes, where the flux condition cannot be posed (the
    // kernel's det = W_f k_s W_s' + c_fs W_s k_f W_f' vanishes): no unknown solid
    // population with a known opposite, and not both an unknown solid population
    // and an unknown fluid population with a known opposite
    long long degen = 0;
    std::vector<uint32_t> words, fb;
    link_words(gs, sm.mask, words, &fb, nullptr);
    static const int O19[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
    static const int O9[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    const int* O = h->p.lattice == MCLBM_D3Q19 ? O19 : O9;
    for (long long q = 0; q < ni; ++q) {
        const uint32_t mf = fb[ibox[(size_t)q]], ms = msb[(size_t)q];
        bool wsp = false, ws = ms != 0, wfp = false;
        for (int i = 1; i < Q; ++i) {
            if (((ms >> i) & 1u) && !((ms >> O[i]) & 1u)) wsp = true;
            if (((mf >> i) & 1u) && !((mf >> O[i]) & 1u)) wfp = true;
        }
        if (!(wsp || (ws && wfp))) ++degen;
    }
    h->nsolid = nsol;
    h->niface = ni;
    h->ndegenerate = degen;
    return MCLBM_OK;
}

// rows per y-band of the fluid numbering: `bands` bands (0: eight, one per
// XCD of a single large lattice), at least 4 rows
static int band_rows(int ny, int bands) {
    const int nb = bands > 0 ? bands : 8;
    return std::max(4, (ny + nb - 1) / nb);
}

static uint32_t tail_link_word(int lattice) {
    const int Q = flow_q(lattice);
    return 0x80000000u | (((1u << Q) - 1u) & ~1u);
}

int mclbm_set_geometry(mclbm_handle* h, const uint8_t* solid_mask, int64_t* n_reclassified) {
    if (!h) return MCLBM_EINVAL;
    if (!solid_mask) return fail(h, MCLBM_EINVAL, "solid_mask is NULL");
    drop_graphs(h);
    h->geom_set = h->fields_set = false;
    int64_t nrc = 0;
    long long kbase = 0;
    std::vector<int> map((size_t)h->Ntot, -1);
    std::vector<unsigned> pos;
    std::vector<uint32_t> links;
    std::vector<int> chunk_sample;
    std::vector<SampleDev> sd(h->S);
    for (int s = 0; s < h->S; ++s) {
        SampleHost& sm = h->smp[s];
        sm.mask.assign(solid_mask + sm.dbase, solid_mask + sm.dbase + sm.N);
        for (auto& m : sm.mask) m = m ? 1 : 0;
        GeomSpec gs{h->p.lattice, sm.nx, sm.ny, sm.nz, h->p.solute};
        nrc += pinch_fill(gs, sm.mask);
        std::vector<uint32_t> words;
        link_words(gs, sm.mask, words, nullptr, nullptr);
        // fluid numbering: y-bands of band_rows(ny) rows, each swept plane by
        // plane (z), row by row, x fastest.  Within a band the nodes of the
        // planes above and below are a few dozen chunks away, so the
        // neighbour gathers of the collide pass (pseudo-potentials, fluid
        // indices) and its pushes across planes stay in the L2 cache of the
        // XCD that sweeps the band.
        sm.pos.clear();
        const int rows = band_rows(sm.ny, h->bands);
        for (int y0 = 0; y0 < sm.ny; y0 += rows)
            for (int z = 0; z < sm.nz; ++z)
                for (int y = y0; y < std::min(sm.ny, y0 + rows); ++y)
                    for (int x = 0; x < sm.nx; ++x) {
                        const long long n = x + (long long)sm.nx * (y + (long long)sm.ny * z);
                        if (sm.mask[n]) continue;
                        map[(size_t)(sm.dbase + n)] = (int)(kbase + (long long)sm.pos.size());
                        sm.pos.push_back((unsigned)n);
                    }
        sm.nf = (long long)sm.pos.size();
        if (sm.nf == 0) {
            char buf[96];
            snprintf(buf, sizeof buf, "sample %d has no fluid node left after reclassification", s);
            return fail(h, MCLBM_EINVAL, buf);
        }
        sm.kbase = kbase;
        const long long padded = pad64(sm.nf);
        pos.resize((size_t)(kbase + padded), 0u);
        // tail lanes of the last chunk: box node 0 of the sample, every flow
        // link blocked and the solid flag (the step kernel has no tail check)
        links.resize((size_t)(kbase + padded), tail_link_word(h->p.lattice));
        for (long long k = 0; k < sm.nf; ++k) {
            pos[(size_t)(kbase + k)] = sm.pos[k];
            links[(size_t)(kbase + k)] = words[sm.pos[k]];
        }
        if (h->dep) {   // deposition updates the geometry incrementally from these
            sm.words.resize((size_t)sm.nf);
            for (long long k = 0; k < sm.nf; ++k) sm.words[(size_t)k] = words[sm.pos[k]];
        }
        for (long long c = 0; c < padded / 64; ++c) chunk_sample.push_back(s);
        sd[s] = SampleDev{sm.nx, sm.ny, sm.nz, (int)sm.nf, (int)sm.N, (int)sm.dbase, (int)sm.kbase, 0};
        sm.frozen = false;
        sm.conv_step = -1;
        sm.div_step = -1;
        sm.bad = false;
        kbase += padded;
    }
    h->nchunks = kbase / 64;
    if (n_reclassified) *n_reclassified = nrc;
    HIPCHK(h, hipMemcpyAsync(h->map, map.data(), map.size() * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->pos, pos.data(), pos.size() * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->links, links.data(), links.size() * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->smp_dev, sd.data(), sd.size() * sizeof(SampleDev), hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->chunk_sample, chunk_sample.data(), chunk_sample.size() * 4, hipMemcpyHostToDevice,
                             h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    int rc = upload_work(h);
    if (rc != MCLBM_OK) return rc;
    h->geom_set = true;
    if (h->dep) {   // no deposit yet
        HIPCHK(h, hipMemsetAsync(h->dep, 0, (size_t)h->nchunks * 64 * 8, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        h->dep_converted = 0;
    }
    if (h->kfield) {   // the rate field starts uniform at k_wall
        std::vector<double> kb((size_t)h->Ntot, h->p.k_wall);
        rc = mclbm_set_wall_rate(h, kb.data());
        if (rc != MCLBM_OK) return rc;
    }
    if (h->thermal) {
        rc = build_thermal(h, map);
        if (rc != MCLBM_OK) {
            h->geom_set = false;
            return rc;
        }
    }
    return MCLBM_OK;
}

int mclbm_set_wall_rate(mclbm_handle* h, const double* k_box) {
    if (!h) return MCLBM_EINVAL;
    if (!h->kfield) return fail(h, MCLBM_ESTATE, "the lattice was created without rate_field");
    if (!h->geom_set) return fail(h, MCLBM_ESTATE, "set_geometry has not been called");
    if (!k_box) return fail(h, MCLBM_EINVAL, "k_box is NULL");
    // stored per fluid node as the two factors the wall rule uses (plane 0: the
    // reacting species' 1 / (2 W + k tau_d / (tau_d - 1/2)), plane 1: the product's
    // gain k tau_d2 / (tau_d2 - 1/2)), in the kernels' arithmetic type
    const size_t M = (size_t)h->nchunks * 64;
    const bool dbl = h->p.storage == MCLBM_F64;
    const int QS = h->QS;
    const double Ws = (1.0 - h->p.J0) / (double)(QS - 1), cs2s = 2.0 * Ws;
    const double tau_d = h->p.D / cs2s + 0.5;
    const double tau_d2 = (h->p.D2 > 0 ? h->p.D2 : 1.0) / cs2s + 0.5;
    std::vector<double> kv(2 * M, 0.0);
    for (const auto& sm : h->smp)
        for (long long k = 0; k < sm.nf; ++k) {
            const double v = k_box[sm.dbase + sm.pos[k]];
            if (!(v >= 0) || !isfinite(v)) return fail(h, MCLBM_EINVAL, "reaction rates must be >= 0 and finite");
            kv[(size_t)(sm.kbase + k)] = 1.0 / (2.0 * Ws + v * tau_d / (tau_d - 0.5));
            kv[M + (size_t)(sm.kbase + k)] = v * tau_d2 / (tau_d2 - 0.5);
        }
    if (dbl) {
        HIPCHK(h, hipMemcpyAsync(h->kfield, kv.data(), 2 * M * 8, hipMemcpyHostToDevice, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
    } else {
        std::vector<float> kf(kv.begin(), kv.end());
        HIPCHK(h, hipMemcpyAsync(h->kfield, kf.data(), 2 * M * 4, hipMemcpyHostToDevice, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
    }
    drop_graphs(h);
    if (h->dep) h->k_box.assign(k_box, k_box + h->Ntot);   // re-applied when deposition rebuilds the geometry
    return MCLBM_OK;
}

int mclbm_get_geometry(mclbm_handle* h, uint8_t* mask_out, uint32_t* flow_links, uint32_t* solute_links) {
    if (!h) return MCLBM_EINVAL;
    if (!h->geom_set) return fail(h, MCLBM_ESTATE, "set_geometry has not been called");
    for (auto& sm : h->smp) {
        if (mask_out) memcpy(mask_out + sm.dbase, sm.mask.data(), (size_t)sm.N);
        if (flow_links || solute_links) {
            std::vector<uint32_t> words, fb, sb;
            GeomSpec gs{h->p.lattice, sm.nx, sm.ny, sm.nz, h->p.solute};
            link_words(gs, sm.mask, words, &fb, &sb);
            if (flow_links) memcpy(flow_links + sm.dbase, fb.data(), (size_t)sm.N * 4);
            if (solute_links) memcpy(solute_links + sm.dbase, sb.data(), (size_t)sm.N * 4);
        }
    }
    return MCLBM_OK;
}

int mclbm_init_fields(mclbm_handle* h, const double* rho, const double* u, const double* C) {
    if (!h) return MCLBM_EINVAL;
    if (!h->geom_set) return fail(h, MCLBM_ESTATE, "set_geometry has not been called");
    if (!rho) return fail(h, MCLBM_EINVAL, "rho is NULL");
    drop_graphs(h);
    long long nf_tot = 0;
    for (auto& sm : h->smp) nf_tot += sm.nf;
    for (int s = 0; s < h->NC; ++s) {
        double sum = 0.0;
        for (auto& sm : h->smp) {
            const double* r = rho + (size_t)h->NC * sm.dbase + (size_t)s * sm.N;
            for (long long n = 0; n < sm.N; ++n) {
                if (sm.mask[n]) continue;
                if (!(r[n] > 0.0) || !isfinite(r[n]))
                    return fail(h, MCLBM_EINVAL, "rho must be > 0 and finite on fluid nodes");
                sum += r[n];
            }
        }
        h->rhobar[s] = sum / (double)nf_tot;
    }
    const long long N = h->Ntot;
    double* st_rho = h->stage;
    double* st_u = h->stage + (size_t)h->NC * N;
    double* st_C = h->stage + (size_t)(h->NC + 3) * N;
    HIPCHK(h, hipMemcpyAsync(st_rho, rho, (size_t)h->NC * N * 8, hipMemcpyHostToDevice, h->stream));
    if (u) HIPCHK(h, hipMemcpyAsync(st_u, u, (size_t)3 * N * 8, hipMemcpyHostToDevice, h->stream));
    if (C && h->p.solute) HIPCHK(h, hipMemcpyAsync(st_C, C, (size_t)N * 8, hipMemcpyHostToDevice, h->stream));
    for (auto& sm : h->smp) {
        sm.frozen = false;
        sm.conv_step = -1;
        sm.div_step = -1;
        sm.bad = false;
        for (int k = 0; k < 16; ++k) sm.mon[k] = 0.0;
        sm.mon[0] = -1.0;
    }
    int rc = upload_work(h);
    if (rc != MCLBM_OK) return rc;
    Ctx c = make_ctx(h);
    HIPCHK(h, k_init(c, st_rho, u ? st_u : nullptr, (C && h->p.solute) ? st_C : nullptr));
    if (h->dep) HIPCHK(h, hipMemsetAsync(h->dep, 0, (size_t)h->nchunks * 64 * 8, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->dep_converted = 0;
    h->step = 0;
    h->snap_valid = false;
    for (int k = 0; k < 16; ++k) h->mon[k] = 0.0;
    h->mon[0] = -1.0;
    h->fields_set = true;
    h->temp_set = false;
    return MCLBM_OK;
}

// The nodes whose deposit exceeds 1 turn solid.  The host updates the geometry
// incrementally (the pinch rule from the new solid nodes, the fluid list in the
// same band order without them, the link words within two nodes of them: the
// same result as mclbm_set_geometry on the new mask) and uploads it; the state
// of every node that is still fluid moves to its new fluid index on the device.
static int convert_deposits(mclbm_handle* h) {
    SampleHost& sm = h->smp[0];   // deposition runs on a single lattice (kbase 0)
    const long long nf_before = sm.nf;
    std::vector<double> dv((size_t)sm.nf);
    HIPCHK(h, hipMemcpyAsync(dv.data(), h->dep, dv.size() * 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    std::vector<long long> add;
    for (long long k = 0; k < sm.nf; ++k)
        if (dv[(size_t)k] > 1.0) add.push_back((long long)sm.pos[k]);
    drop_graphs(h);
    const GeomSpec gs{h->p.lattice, sm.nx, sm.ny, sm.nz, h->p.solute};
    std::vector<int> from;
    convert_nodes(gs, sm.mask, sm.pos, sm.words, add, from);
    sm.nf = (long long)sm.pos.size();
    if (sm.nf == 0) {
        h->geom_set = h->fields_set = false;
        return fail(h, MCLBM_EINVAL, "deposition left no fluid node (the lattice needs set_geometry again)");
    }
    // device geometry in the new numbering (tail lanes as set_geometry makes them)
    const long long padded = pad64(sm.nf);
    std::vector<int> map((size_t)h->Ntot, -1);
    std::vector<unsigned> pos((size_t)padded, 0u);
    std::vector<uint32_t> links((size_t)padded, tail_link_word(h->p.lattice));
    std::vector<int> fromp((size_t)padded, -1);
    std::vector<double> dn((size_t)padded, 0.0);
    for (long long k = 0; k < sm.nf; ++k) {
        map[sm.pos[k]] = (int)k;
        pos[(size_t)k] = sm.pos[k];
        links[(size_t)k] = sm.words[(size_t)k];
        fromp[(size_t)k] = from[(size_t)k];
        dn[(size_t)k] = dv[(size_t)from[(size_t)k]];
    }
    const std::vector<int> chunk_sample((size_t)(padded / 64), 0);
    const SampleDev sd{sm.nx, sm.ny, sm.nz, (int)sm.nf, (int)sm.N, (int)sm.dbase, (int)sm.kbase, 0};
    h->nchunks = padded / 64;
    HIPCHK(h, hipMemcpyAsync(h->map, map.data(), map.size() * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->pos, pos.data(), pos.size() * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->links, links.data(), links.size() * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->smp_dev, &sd, sizeof(SampleDev), hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->chunk_sample, chunk_sample.data(), chunk_sample.size() * 4, hipMemcpyHostToDevice,
                             h->stream));
    // the state moves to the new numbering on the device (the batch snapshot area
    // is free here and holds at least M doubles)
    int* d_from = (int*)h->dep_snap;
    HIPCHK(h, hipMemcpyAsync(d_from, fromp.data(), fromp.size() * 4, hipMemcpyHostToDevice, h->stream));
    const int sb = (int)store_bytes(h->p.storage);
    // paired 16-bit flow storage moves as Q planes of 32-bit words
    if (flow_pairs(h))
        HIPCHK(h, k_remap_planes(h->fB, h->fA, h->Q, d_from, padded, 2 * sb, h->stream));
    else
        HIPCHK(h, k_remap_planes(h->fB, h->fA, h->NC * h->Q, d_from, padded, sb, h->stream));
    std::swap(h->fA, h->fB);
    HIPCHK(h, k_remap_planes(h->hB, h->hA, h->HP, d_from, padded, sb, h->stream));
    std::swap(h->hA, h->hB);
    HIPCHK(h, hipMemcpyAsync(h->dep, dn.data(), dn.size() * 8, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));   // before the host vectors go
    int rc = upload_work(h);
    if (rc != MCLBM_OK) return rc;
    if (h->kfield) {   // the rate planes follow the new numbering
        const std::vector<double> kb = h->k_box;
        rc = mclbm_set_wall_rate(h, kb.data());
        if (rc != MCLBM_OK) return rc;
    }
    h->snap_valid = false;
    h->dep_converted += nf_before - sm.nf;
    return MCLBM_OK;
}

int mclbm_get_deposit(mclbm_handle* h, double* Cps, int64_t* converted) {
    if (!h) return MCLBM_EINVAL;
    if (!h->dep) return fail(h, MCLBM_EINVAL, "the lattice was created without deposition");
    if (!h->fields_set) return fail(h, MCLBM_ESTATE, "init_fields has not been called");
    if (Cps) {
        const SampleHost& sm = h->smp[0];
        std::vector<double> dv((size_t)sm.nf);
        HIPCHK(h, hipMemcpyAsync(dv.data(), h->dep + sm.kbase, dv.size() * 8, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        memset(Cps, 0, (size_t)sm.N * 8);
        for (long long k = 0; k < sm.nf; ++k) Cps[sm.pos[k]] = dv[(size_t)k];
    }
    if (converted) *converted = h->dep_converted;
    return MCLBM_OK;
}

// Steps with particle deposition (eq:surface_deposition).  Steps run in batches
// of up to DEP_BATCH, never past the next monitor step.  Each step is followed
// by the deposit update, which counts the deposits above 1 into a slot of its
// own, and one synchronisation per batch reads the counts.  The populations and
// deposits at the start of the batch are kept in a device snapshot: if the j-th
// step of the batch made some deposit exceed 1 and later steps ran on, the
// snapshot is restored and the first j steps are run again (every value these
// kernels write is deterministic; the count is the only atomic), so the state
// is reproduced bit for bit; those nodes then turn solid before the next step.
// The batch length adapts to the spacing of conversions (twice the steps to the
// last one, doubled after a batch without one), so that dense conversions do
// not waste most of a long batch.
static int step_deposition(mclbm_handle* h, int64_t n) {
    const int K = h->p.monitor_every;
    const size_t sb = store_bytes(h->p.storage);
    bool monitored = false, had = false;
    int64_t left = n;
    while (left > 0) {
        const int64_t to_monitor = K - (h->step % K);
        const int B = (int)std::min(std::min(left, (int64_t)h->dep_batch), to_monitor);
        const size_t M = (size_t)h->nchunks * 64;
        const size_t fbytes = (size_t)h->NC * h->Q * M * sb, hbytes = (size_t)h->HP * M * sb;
        char* snap = (char*)h->dep_snap;
        if (B > 1) {
            HIPCHK(h, hipMemcpyAsync(snap, h->fA, fbytes, hipMemcpyDeviceToDevice, h->stream));
            HIPCHK(h, hipMemcpyAsync(snap + fbytes, h->hA, hbytes, hipMemcpyDeviceToDevice, h->stream));
            HIPCHK(h, hipMemcpyAsync(snap + fbytes + hbytes, h->dep, M * 8, hipMemcpyDeviceToDevice, h->stream));
        }
        const int64_t step0 = h->step;
        HIPCHK(h, hipMemsetAsync(h->dep_count, 0, DEP_BATCH * 4, h->stream));
        for (int j = 0; j < B; ++j) {
            int rc = launch_step(h, h->stream);
            if (rc != MCLBM_OK) return rc;
            HIPCHK(h, k_deposit_step(make_ctx(h), h->dep, h->p.dep_prob, h->dep_count + j));
        }
        HIPCHK(h, hipMemcpyAsync(h->host_dep, h->dep_count, (size_t)B * 4, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        int first = -1;
        for (int j = 0; j < B && first < 0; ++j)
            if (h->host_dep[j] > 0) first = j;
        if (first < 0) {
            left -= B;
            h->dep_batch = std::min(DEP_BATCH, 2 * h->dep_batch);
        } else {
            h->dep_batch = std::min(DEP_BATCH, 2 * (first + 1));
            if (first < B - 1) {   // back to the start of the batch, then up to the crossing step
                HIPCHK(h, hipMemcpyAsync(h->fA, snap, fbytes, hipMemcpyDeviceToDevice, h->stream));
                HIPCHK(h, hipMemcpyAsync(h->hA, snap + fbytes, hbytes, hipMemcpyDeviceToDevice, h->stream));
                HIPCHK(h, hipMemcpyAsync(h->dep, snap + fbytes + hbytes, M * 8, hipMemcpyDeviceToDevice, h->stream));
                h->step = step0;
                for (int j = 0; j <= first; ++j) {
                    int rc = launch_step(h, h->stream);
                    if (rc != MCLBM_OK) return rc;
                    HIPCHK(h, k_deposit_step(make_ctx(h), h->dep, h->p.dep_prob, h->dep_count + j));
                }
            }
            int rc = convert_deposits(h);
            if (rc != MCLBM_OK) return rc;
            left -= first + 1;
        }
        if (h->step % K == 0) {
            had = h->snap_valid;
            HIPCHK(h, k_monitor(make_ctx(h), had ? 1 : 0));
            h->snap_valid = true;
            monitored = true;
        }
    }
    if (monitored) return collect_monitor(h, had);
    return MCLBM_OK;
}

int mclbm_set_deposit(mclbm_handle* h, const double* Cps, int64_t converted) {
    if (!h) return MCLBM_EINVAL;
    if (!h->dep) return fail(h, MCLBM_EINVAL, "the lattice was created without deposition");
    if (!h->fields_set) return fail(h, MCLBM_ESTATE, "init_fields has not been called");
    if (!Cps) return fail(h, MCLBM_EINVAL, "Cps is NULL");
    if (converted < 0) return fail(h, MCLBM_EINVAL, "converted must be >= 0");
    const SampleHost& sm = h->smp[0];
    std::vector<double> dv((size_t)sm.nf);
    for (long long k = 0; k < sm.nf; ++k) {
        const double v = Cps[sm.pos[k]];
        if (!(v >= 0) || !isfinite(v)) return fail(h, MCLBM_EINVAL, "deposits must be >= 0 and finite");
        dv[(size_t)k] = v;
    }
    HIPCHK(h, hipMemcpyAsync(h->dep, dv.data(), dv.size() * 8, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->dep_converted = converted;
    return MCLBM_OK;
}

int mclbm_step(mclbm_handle* h, int64_t n) {
    if (!h) return MCLBM_EINVAL;
    if (n < 0) return fail(h, MCLBM_EINVAL, "n must be >= 0");
    if (!h->fields_set) return fail(h, MCLBM_ESTATE, "init_fields has not been called");
    if (h->thermal && !h->temp_set) return fail(h, MCLBM_ESTATE, "init_temperature has not been called");
    if (h->dep) return step_deposition(h, n);
    const int K = h->p.monitor_every;
    bool monitored = false, had = false;
    int64_t left = n;
    while (left > 0) {
        // a whole aligned interval through the graph when possible
        if (h->use_graph && h->snap_valid && (K % 2 == 0) && h->step % K == 0 && left >= K) {
            int rc = replay_interval(h);
            if (rc != MCLBM_OK) return rc;
            left -= K;
            had = true;
            monitored = true;
            continue;
        }
        int rc = launch_step(h, h->stream);
        if (rc != MCLBM_OK) return rc;
        --left;
        if (h->step % K == 0) {
            had = h->snap_valid;
            HIPCHK(h, k_monitor(make_ctx(h), had ? 1 : 0));
            h->snap_valid = true;
            monitored = true;
        }
    }
    if (monitored) return collect_monitor(h, had);
    return MCLBM_OK;
}

int mclbm_monitor_now(mclbm_handle* h) {
    if (!h) return MCLBM_EINVAL;
    if (!h->fields_set) return fail(h, MCLBM_ESTATE, "init_fields has not been called");
    const bool had = h->snap_valid;
    HIPCHK(h, k_monitor(make_ctx(h), had ? 1 : 0));
    h->snap_valid = true;
    return collect_monitor(h, had);
}

int mclbm_get_moments(mclbm_handle* h, double* rho, double* u, double* C, int32_t dst_is_device) {
    if (!h) return MCLBM_EINVAL;
    if (!h->fields_set) return fail(h, MCLBM_ESTATE, "init_fields has not been called");
    Ctx c = make_ctx(h);
    const long long N = h->Ntot;
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
    const size_t nsp = (h->p.solute && h->p.product) ? 2 : 1;   // C: [species][N] per sample
    if (C) HIPCHK(h, hipMemcpyAsync(C, st_C, nsp * (size_t)N * 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return MCLBM_OK;
}

int mclbm_get_monitors(mclbm_handle* h, double out[16]) {
    if (!h || !out) return MCLBM_EINVAL;
    for (int k = 0; k < 16; ++k) out[k] = h->mon[k];
    out[10] = (double)h->step;
    return MCLBM_OK;
}

int mclbm_get_sample_monitors(mclbm_handle* h, int32_t s, double out[16]) {
    if (!h || !out) return MCLBM_EINVAL;
    if (s < 0 || s >= h->S) return fail(h, MCLBM_EINVAL, "sample index out of range");
    for (int k = 0; k < 16; ++k) out[k] = h->smp[s].mon[k];
    out[10] = (double)h->step;
    out[11] = (double)h->smp[s].conv_step;
    out[12] = h->smp[s].frozen ? 1.0 : 0.0;
    out[13] = (double)h->smp[s].div_step;
    return MCLBM_OK;
}

int mclbm_population_bytes(mclbm_handle* h, int32_t raw, size_t* bytes) {
    if (!h || !bytes) return MCLBM_EINVAL;
    const size_t nval = (size_t)(h->NC * h->Q + h->HP) * (size_t)h->Ntot;
    *bytes = nval * (raw ? store_bytes(h->p.storage) : 8);
    return MCLBM_OK;
}

int mclbm_get_populations(mclbm_handle* h, void* dst, int32_t raw) {
    if (!h || !dst) return MCLBM_EINVAL;
    if (!h->fields_set) return fail(h, MCLBM_ESTATE, "init_fields has not been called");
    const size_t sb = store_bytes(h->p.storage);
    const size_t M = (size_t)h->nchunks * 64;
    const size_t PF = (size_t)h->NC * h->Q, PS = (size_t)h->HP;
    std::vector<unsigned char> dev((PF + PS) * M * sb);
    HIPCHK(h, hipMemcpyAsync(dev.data(), h->fA, PF * M * sb, hipMemcpyDeviceToHost, h->stream));
    if (PS) HIPCHK(h, hipMemcpyAsync(dev.data() + PF * M * sb, h->hA, PS * M * sb, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    const Ctx c = make_ctx(h);
    const size_t nplanes = PF + PS, ob = raw ? sb : 8;
    memset(dst, 0, nplanes * (size_t)h->Ntot * ob);
    for (auto& sm : h->smp) {
        const size_t N = (size_t)sm.N;
        unsigned char* out = (unsigned char*)dst + nplanes * (size_t)sm.dbase * ob;
        for (size_t j = 0; j < nplanes; ++j) {
            const bool flow = j < PF;
            const unsigned char* src = flow ? dev.data() : dev.data() + PF * M * sb;
            const size_t P = flow ? PF : PS, jj = flow ? j : j - PF;
            const int s = flow ? (int)(j / h->Q) : 0, i = flow ? (int)(j % h->Q) : 0;
            const float shift = flow ? shift_f32(c, s, i) : 0.0f;
            for (size_t k = 0; k < (size_t)sm.nf; ++k) {
                const size_t q = flow ? flow_index(h, j, (size_t)sm.kbase + k) : blk_index(P, jj, (size_t)sm.kbase + k);
                const size_t o = j * N + sm.pos[k];
                if (raw) {
                    memcpy(out + o * sb, src + q * sb, sb);
                    continue;
                }
                double v;
                switch (h->p.storage) {
                    case MCLBM_F64: v = ((const double*)src)[q]; break;
                    case MCLBM_F32: v = ((const float*)src)[q]; break;
                    case MCLBM_F16_SHIFT: v = (double)(half_to_float(((const uint16_t*)src)[q]) + shift); break;
                    default: v = (double)(bf16_to_float_h(((const uint16_t*)src)[q]) + shift); break;
                }
                ((double*)out)[o] = v;
            }
        }
    }
    return MCLBM_OK;
}

int mclbm_set_populations(mclbm_handle* h, const void* src, int32_t raw) {
    if (!h || !src) return MCLBM_EINVAL;
    if (!h->fields_set) return fail(h, MCLBM_ESTATE, "init_fields has not been called");
    const size_t sb = store_bytes(h->p.storage);
    const size_t M = (size_t)h->nchunks * 64;
    const size_t PF = (size_t)h->NC * h->Q, PS = (size_t)h->HP;
    const size_t nplanes = PF + PS, ib = raw ? sb : 8;
    // raw: the stored bytes are copied as they are; otherwise the FP64 values
    // are laid out in the chunked order and encoded on the device by the same
    // store the step kernels use
    const size_t eb = raw ? sb : 8;
    std::vector<unsigned char> dev((PF + PS) * M * eb, 0);
    const Ctx c = make_ctx(h);
    for (auto& sm : h->smp) {
        const size_t N = (size_t)sm.N;
        const unsigned char* in = (const unsigned char*)src + nplanes * (size_t)sm.dbase * ib;
        for (size_t j = 0; j < nplanes; ++j) {
            const bool flow = j < PF;
            unsigned char* dstp = flow ? dev.data() : dev.data() + PF * M * eb;
            const size_t P = flow ? PF : PS, jj = flow ? j : j - PF;
            for (size_t k = 0; k < (size_t)sm.nf; ++k) {
                const size_t q = flow ? flow_index(h, j, (size_t)sm.kbase + k) : blk_index(P, jj, (size_t)sm.kbase + k);
                const size_t o = j * N + sm.pos[k];
                memcpy(dstp + q * eb, in + o * eb, eb);
            }
        }
    }
    if (raw) {
        HIPCHK(h, hipMemcpyAsync(h->fA, dev.data(), PF * M * sb, hipMemcpyHostToDevice, h->stream));
        if (PS)
            HIPCHK(h, hipMemcpyAsync(h->hA, dev.data() + PF * M * sb, PS * M * sb, hipMemcpyHostToDevice, h->stream));
    } else {
        // pieces of at most the staging capacity, FP64 in, storage format out
        const long long cap = (long long)((size_t)(h->NC + 4) * (size_t)h->Ntot);
        const double* hv = (const double*)dev.data();
        for (int arr = 0; arr < (PS ? 2 : 1); ++arr) {
            const long long tot = (long long)((arr ? PS : PF) * M);
            const double* base = hv + (arr ? PF * M : 0);
            void* dst = arr ? h->hA : h->fA;
            for (long long q0 = 0; q0 < tot; q0 += cap) {
                const long long cnt = std::min(cap, tot - q0);
                HIPCHK(h, hipMemcpyAsync(h->stage, base + q0, (size_t)cnt * 8, hipMemcpyHostToDevice, h->stream));
                HIPCHK(h, k_encode_planes(c, h->stage, dst, q0, cnt, (int)(arr ? PS : PF), arr ? 0 : 1));
            }
        }
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    // a new state for every sample: convergence flags (frozen samples would
    // otherwise keep a stale mirror in B) and the residual snapshot start over
    drop_graphs(h);
    h->snap_valid = false;
    for (auto& sm : h->smp) {
        sm.frozen = false;
        sm.conv_step = -1;
        sm.div_step = -1;
        sm.bad = false;
    }
    return upload_work(h);
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
        if (e != MCLBM_OK && e != MCLBM_EDIVERGED) {
            if (steps_taken) *steps_taken = taken;
            return e;
        }
        if (h->step % K != 0) continue;
        bool active = false, changed = false, any_div = false;
        for (auto& sm : h->smp) {
            if (sm.frozen) {
                any_div |= sm.div_step >= 0;
                continue;
            }
            const bool fresh = sm.mon[0] == (double)h->step;
            if (fresh && sm.bad) {
                sm.frozen = true;
                sm.div_step = h->step;
                sm.mon[12] = 1.0;
                changed = any_div = true;
            } else if (fresh && sm.mon[9] <= tol) {
                sm.frozen = true;
                sm.conv_step = h->step;
                sm.mon[11] = (double)sm.conv_step;
                sm.mon[12] = 1.0;
                changed = true;
                if (h->S > 1) {
                    int m = mirror_sample(h, sm);
                    if (m != MCLBM_OK) return m;
                }
            } else {
                active = true;
            }
        }
        if (!active) {
            rc = any_div ? fail(h, MCLBM_EDIVERGED, "a sample went non-finite (see the sample monitors)") : MCLBM_OK;
            break;
        }
        // graphs hold grid sizes and the work-list choice: capture again
        if (changed) drop_graphs(h);
        if (changed) {
            int u = upload_work(h);
            if (u != MCLBM_OK) return u;
        }
    }
    if (steps_taken) *steps_taken = taken;
    return rc;
}

int mclbm_set_launch(mclbm_handle* h, int32_t block_threads, int32_t grid_blocks) {
    if (!h) return MCLBM_EINVAL;
    if (block_threads != 64 && block_threads != 128 && block_threads != 256)
        return fail(h, MCLBM_EINVAL, "block_threads must be 64, 128 or 256");
    if (grid_blocks < 0 || (grid_blocks % 8) != 0)
        return fail(h, MCLBM_EINVAL, "grid_blocks must be 0 or a positive multiple of 8");
    drop_graphs(h);
    h->block = block_threads;
    h->grid = grid_blocks;
    return MCLBM_OK;
}

int mclbm_set_addressing(mclbm_handle* h, int32_t flat) {
    if (!h) return MCLBM_EINVAL;
    if (flat != 0 && flat != 1) return fail(h, MCLBM_EINVAL, "flat must be 0 or 1");
    drop_graphs(h);
    h->flat = flat;
    return MCLBM_OK;
}

// Numbers the fluid nodes again with the current band count: set_geometry on
// the current (reclassified) masks of every sample.
static int renumber(mclbm_handle* h) {
    std::vector<uint8_t> mask((size_t)h->Ntot, 0);
    for (auto& sm : h->smp) std::copy(sm.mask.begin(), sm.mask.end(), mask.begin() + sm.dbase);
    return mclbm_set_geometry(h, mask.data(), nullptr);
}

int mclbm_set_bands(mclbm_handle* h, int32_t bands) {
    if (!h) return MCLBM_EINVAL;
    if (bands < 0 || bands > 64) return fail(h, MCLBM_EINVAL, "bands must be 0 (eight) or 1 .. 64");
    if (bands == h->bands) return MCLBM_OK;
    h->bands = bands;
    return h->geom_set ? renumber(h) : MCLBM_OK;
}

int mclbm_autotune(mclbm_handle* h, int32_t trial_steps, int32_t* bands, int32_t* block_threads,
                   int32_t* grid_blocks, double* ms_per_step, double* table, int32_t table_rows, int32_t* n_rows) {
    if (!h) return MCLBM_EINVAL;
    if (!h->geom_set) return fail(h, MCLBM_ESTATE, "set_geometry has not been called");
    if (trial_steps < 1) return fail(h, MCLBM_EINVAL, "trial_steps must be >= 1");
    int dev = 0, cus = 0;
    HIPCHK(h, hipGetDevice(&dev));
    HIPCHK(h, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    // band counts: the current one first; the others only where numbering the
    // fluid nodes again loses no caller state (rate field, deposits, heat)
    const int old_bands = h->bands;
    std::vector<int> band_cand{old_bands};
    if (!h->kfield && !h->dep && !h->thermal)
        for (int nb : {0, 4, 16})
            if (nb != old_bands) band_cand.push_back(nb);
    std::vector<std::pair<int, int>> shapes;
    for (int b : {64, 128, 256}) {
        shapes.push_back({b, 0});
        for (int w : {8, 16, 32}) {
            const int g = (cus * w / (b / 64) + 7) / 8 * 8;
            if (g > 0) shapes.push_back({b, g});
        }
    }
    hipEvent_t e0, e1;
    HIPCHK(h, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(h, MCLBM_EHIP, "hipEventCreate failed");
    }
    const int old_block = h->block, old_grid = h->grid;
    double best = INFINITY;
    int bn = old_bands, bb = old_block, bg = old_grid, rc = MCLBM_OK;
    size_t row = 0;
    for (size_t bi = 0; bi < band_cand.size() && rc == MCLBM_OK; ++bi) {
        if (band_cand[bi] != h->bands) {
            h->bands = band_cand[bi];
            rc = renumber(h);
            if (rc != MCLBM_OK) break;
        }
        {
            std::vector<double> rho((size_t)h->NC * h->Ntot, 1.0);
            rc = mclbm_init_fields(h, rho.data(), nullptr, nullptr);
            if (rc != MCLBM_OK) break;
        }
        for (size_t i = 0; i < shapes.size() && rc == MCLBM_OK; ++i, ++row) {
            h->block = shapes[i].first;
            h->grid = shapes[i].second;
            for (int s = 0; s < 2 && rc == MCLBM_OK; ++s) rc = launch_step(h, h->stream);
            if (rc != MCLBM_OK) break;
            hipError_t e = hipEventRecord(e0, h->stream);
            for (int s = 0; s < trial_steps && rc == MCLBM_OK && e == hipSuccess; ++s) rc = launch_step(h, h->stream);
            if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess && rc == MCLBM_OK) rc = hip_fail(h, e, "autotune timing");
            if (rc != MCLBM_OK) break;
            const double per = (double)ms / trial_steps;
            if (table && (int)row < table_rows) {
                table[4 * row + 0] = band_cand[bi];
                table[4 * row + 1] = shapes[i].first;
                table[4 * row + 2] = shapes[i].second;
                table[4 * row + 3] = per;
            }
            if (per < best) {
                best = per;
                bn = band_cand[bi];
                bb = shapes[i].first;
                bg = shapes[i].second;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == MCLBM_OK && h->bands != bn) {
        h->bands = bn;
        rc = renumber(h);
    }
    h->fields_set = false;
    h->step = 0;
    h->snap_valid = false;
    drop_graphs(h);
    if (rc != MCLBM_OK) {
        h->block = old_block;
        h->grid = old_grid;
        return rc;
    }
    h->block = bb;
    h->grid = bg;
    if (bands) *bands = bn;
    if (block_threads) *block_threads = bb;
    if (grid_blocks) *grid_blocks = bg;
    if (ms_per_step) *ms_per_step = best;
    if (n_rows) *n_rows = (int32_t)row;
    return MCLBM_OK;
}

int mclbm_set_graph(mclbm_handle* h, int32_t enable) {
    if (!h) return MCLBM_EINVAL;
    if (enable && (h->p.monitor_every % 2) != 0)
        return fail(h, MCLBM_EINVAL, "graph replay needs an even monitor_every");
    drop_graphs(h);
    h->use_graph = enable != 0;
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

int mclbm_set_thermal(mclbm_handle* h, const mclbm_thermal* t) {
    if (!h) return MCLBM_EINVAL;
    if (!t) return fail(h, MCLBM_EINVAL, "thermal parameters are NULL");
    if (h->S != 1) return fail(h, MCLBM_EINVAL, "conjugate heat transfer needs a single lattice");
    if (h->p.storage != MCLBM_F64 && h->p.storage != MCLBM_F32)
        return fail(h, MCLBM_EINVAL, "conjugate heat transfer needs F64 or F32 storage");
    if (h->p.deposition || h->p.rate_field)
        return fail(h, MCLBM_EINVAL, "conjugate heat transfer excludes deposition and rate_field");
    auto pos = [](double v) { return v > 0 && isfinite(v); };
    auto nonneg = [](double v) { return v >= 0 && isfinite(v); };
    if (!(t->tau_ef > 0.5) || !isfinite(t->tau_ef) || !(t->tau_es > 0.5) || !isfinite(t->tau_es))
        return fail(h, MCLBM_EINVAL, "tau_ef and tau_es must be > 1/2");
    if (!pos(t->rhocp_f) || !pos(t->rhocp_s)) return fail(h, MCLBM_EINVAL, "rhocp_f and rhocp_s must be > 0");
    if (!nonneg(t->h_r) || !nonneg(t->A) || !nonneg(t->E_over_R))
        return fail(h, MCLBM_EINVAL, "h_r, A and E_over_R must be >= 0 and finite");
    if (!pos(t->T_tol) || t->T_maxit < 1 || t->reserved != 0)
        return fail(h, MCLBM_EINVAL, "T_tol must be > 0, T_maxit >= 1, reserved 0");
    drop_graphs(h);
    free_thermal(h);
    h->th = *t;
    h->thermal = true;
    h->geom_set = h->fields_set = false;
    return MCLBM_OK;
}

int mclbm_init_temperature(mclbm_handle* h, const double* T, const double* u) {
    if (!h) return MCLBM_EINVAL;
    if (!h->thermal) return fail(h, MCLBM_ESTATE, "set_thermal has not been called");
    if (!h->fields_set || !h->gA) return fail(h, MCLBM_ESTATE, "init_fields has not been called");
    if (!T) return fail(h, MCLBM_EINVAL, "T is NULL");
    const long long N = h->Ntot;
    for (long long n = 0; n < N; ++n)
        if (!(T[n] > 0) || !isfinite(T[n])) return fail(h, MCLBM_EINVAL, "T must be > 0 and finite");
    drop_graphs(h);
    double* st_T = h->stage;
    double* st_u = h->stage + N;   // the staging area holds at least (ncomp + 4) N doubles
    HIPCHK(h, hipMemcpyAsync(st_T, T, (size_t)N * 8, hipMemcpyHostToDevice, h->stream));
    if (u) HIPCHK(h, hipMemcpyAsync(st_u, u, (size_t)3 * N * 8, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, k_thermal_init(make_ctx(h), st_T, u ? st_u : nullptr));
    HIPCHK(h, hipMemsetAsync(h->th_stats, 0, 64, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->temp_set = true;
    return MCLBM_OK;
}

int mclbm_get_temperature(mclbm_handle* h, double* T) {
    if (!h) return MCLBM_EINVAL;
    if (!h->thermal || !h->temp_set) return fail(h, MCLBM_ESTATE, "init_temperature has not been called");
    if (!T) return fail(h, MCLBM_EINVAL, "T is NULL");
    const long long N = h->Ntot;
    HIPCHK(h, hipMemsetAsync(h->stage, 0, (size_t)N * 8, h->stream));
    HIPCHK(h, k_thermal_out(make_ctx(h), 0, 0, h->stage));
    HIPCHK(h, hipMemcpyAsync(T, h->stage, (size_t)N * 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return MCLBM_OK;
}

int mclbm_get_thermal_populations(mclbm_handle* h, double* g, double* gs) {
    if (!h) return MCLBM_EINVAL;
    if (!h->thermal || !h->temp_set) return fail(h, MCLBM_ESTATE, "init_temperature has not been called");
    const long long N = h->Ntot;
    for (int which = 1; which <= 2; ++which) {
        double* dst = which == 1 ? g : gs;
        if (!dst) continue;
        for (int i = 0; i < h->Q; ++i) {
            HIPCHK(h, hipMemsetAsync(h->stage, 0, (size_t)N * 8, h->stream));
            HIPCHK(h, k_thermal_out(make_ctx(h), which, i, h->stage));
            HIPCHK(h, hipMemcpyAsync(dst + (size_t)i * N, h->stage, (size_t)N * 8, hipMemcpyDeviceToHost, h->stream));
        }
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return MCLBM_OK;
}

int mclbm_get_thermal_stats(mclbm_handle* h, int64_t out[3]) {
    if (!h) return MCLBM_EINVAL;
    if (!h->thermal || !h->temp_set) return fail(h, MCLBM_ESTATE, "init_temperature has not been called");
    if (!out) return fail(h, MCLBM_EINVAL, "out is NULL");
    unsigned long long st[2] = {0, 0};
    HIPCHK(h, hipMemcpyAsync(st, h->th_stats, sizeof st, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    out[0] = (int64_t)st[0];
    out[1] = (int64_t)st[1];
    out[2] = (int64_t)h->ndegenerate;
    return MCLBM_OK;
}

void mclbm_destroy(mclbm_handle* h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    if (h->gstream) (void)hipStreamSynchronize(h->gstream);
    drop_graphs(h);
    if (h->ev_in) (void)hipEventDestroy(h->ev_in);
    if (h->ev_out) (void)hipEventDestroy(h->ev_out);
    if (h->gstream) (void)hipStreamDestroy(h->gstream);
    if (h->host_result) (void)hipHostFree(h->host_result);
    if (h->host_nwork) (void)hipHostFree(h->host_nwork);
    if (h->host_dep) (void)hipHostFree(h->host_dep);
    if (h->own_arena && h->arena) (void)hipFree(h->arena);
    free_thermal(h);
    delete h;
}

const char* mclbm_last_error(const mclbm_handle* h) {
    if (!h) return g_global_error.c_str();
    return h->err.c_str();
}

}  // extern "C"
