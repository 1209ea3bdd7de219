// Host-side geometry preparation: pinch-fill and per-node link words.
//
// Pinch-fill: a fluid voxel with blocked neighbours on both sides along one
// axis (x, y, and z in 3-D; periodic wrap; in inlet/outlet solute mode the
// planes beyond x = 0 and x = nx-1 count as blocked) has no fluid population
// to reflect at a wet link, so it is made solid.  Making a voxel solid can
// only add pinches, so the result is the least fixed point above the input
// mask whatever the processing order; a work list reaches it in O(N).
#include <stdint.h>

#include <algorithm>
#include <thread>
#include <vector>

#include "geometry.hpp"

namespace mclbm {

namespace {

struct Grid {
    int nx, ny, nz, dim;
    bool seam;
    // periodic wrap of coordinates a few nodes outside the box (no division)
    static int wrap(int a, int n) {
        while (a < 0) a += n;
        while (a >= n) a -= n;
        return a;
    }
    long long idx(int x, int y, int z) const {
        return (long long)wrap(x, nx) + (long long)nx * ((long long)wrap(y, ny) + (long long)ny * wrap(z, nz));
    }
};

bool blocked(const Grid& g, const std::vector<uint8_t>& m, int x, int y, int z) {
    if (g.seam && (x < 0 || x >= g.nx)) return true;
    return m[g.idx(x, y, z)] != 0;
}

bool pinched(const Grid& g, const std::vector<uint8_t>& m, int x, int y, int z) {
    static const int ax[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int a = 0; a < g.dim; ++a)
        if (blocked(g, m, x + ax[a][0], y + ax[a][1], z + ax[a][2]) &&
            blocked(g, m, x - ax[a][0], y - ax[a][1], z - ax[a][2]))
            return true;
    return false;
}

// fn(t, z, y) for every row (z, y) of the box, rows dealt round-robin to up to
// 16 threads (t = thread index)
template <class F>
unsigned parallel_rows(int ny, int nz, F fn) {
    const long long rows = (long long)ny * nz;
    unsigned nt = std::thread::hardware_concurrency();
    if (nt == 0) nt = 1;
    if (nt > 16) nt = 16;
    if ((long long)nt > rows / 64 + 1) nt = (unsigned)(rows / 64 + 1);
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t)
        th.emplace_back([&, t]() {
            for (long long r = t; r < rows; r += nt) fn(t, (int)(r / ny), (int)(r % ny));
        });
    for (auto& x : th) x.join();
    return nt;
}

}  // namespace

int64_t pinch_fill(const GeomSpec& s, std::vector<uint8_t>& mask) {
    Grid g{s.nx, s.ny, s.nz, s.lattice == 1 ? 3 : 2, s.solute == 2};
    // initial scan in parallel (read-only), then the work list in one thread
    std::vector<std::vector<long long>> found(16);
    parallel_rows(g.ny, g.nz, [&](unsigned t, int z, int y) {
        for (int x = 0; x < g.nx; ++x) {
            long long n = g.idx(x, y, z);
            if (!mask[n] && pinched(g, mask, x, y, z)) found[t].push_back(n);
        }
    });
    std::vector<long long> work;
    for (auto& f : found) work.insert(work.end(), f.begin(), f.end());
    int64_t count = 0;
    static const int ax[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    while (!work.empty()) {
        long long n = work.back();
        work.pop_back();
        if (mask[n]) continue;
        mask[n] = 1;
        ++count;
        int x = (int)(n % g.nx), y = (int)((n / g.nx) % g.ny), z = (int)(n / ((long long)g.nx * g.ny));
        for (int a = 0; a < g.dim; ++a)
            for (int sgn = -1; sgn <= 1; sgn += 2) {
                int xx = x + sgn * ax[a][0], yy = y + sgn * ax[a][1], zz = z + sgn * ax[a][2];
                if (g.seam && (xx < 0 || xx >= g.nx)) continue;
                long long m = g.idx(xx, yy, zz);
                xx = (int)(m % g.nx);
                yy = (int)((m / g.nx) % g.ny);
                zz = (int)(m / ((long long)g.nx * g.ny));
                if (!mask[m] && pinched(g, mask, xx, yy, zz)) work.push_back(m);
            }
    }
    return count;
}

// Lattice vectors (paper tables), flow then the solute subset (first QS).
static const int C19[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
                               {1, 1, 0},  {-1, -1, 0}, {1, 0, 1},  {-1, 0, -1}, {0, 1, 1},  {0, -1, -1}, {1, -1, 0},
                               {-1, 1, 0}, {1, 0, -1}, {-1, 0, 1}, {0, 1, -1}, {0, -1, 1}};
static const int C9[9][3] = {{0, 0, 0}, {1, 0, 0},  {0, 1, 0},   {-1, 0, 0}, {0, -1, 0},
                             {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};

namespace {

struct WordCtx {
    Grid g;
    int Q, QS;
    const int (*c)[3];
    int wet_shift, hop_shift;
    bool in_x(int x) const { return !g.seam || (x >= 0 && x < g.nx); }
};

WordCtx word_ctx(const GeomSpec& s) {
    WordCtx w{Grid{s.nx, s.ny, s.nz, s.lattice == 1 ? 3 : 2, s.solute == 2}, s.lattice == 1 ? 19 : 9,
              s.lattice == 1 ? 7 : 5, s.lattice == 1 ? C19 : C9, s.lattice == 1 ? 18 : 8, s.lattice == 1 ? 24 : 12};
    return w;
}

// Link word of the fluid node (x, y, z): upstream-solid flow bits, wet solute
// links, and the bits of the solute directions whose next node is fluid with a
// wet link in that direction.
uint32_t word_at(const WordCtx& W, const std::vector<uint8_t>& mask, int x, int y, int z, uint32_t* fb_out,
                 uint32_t* sb_out) {
    const Grid& g = W.g;
    const int(*c)[3] = W.c;
    uint32_t fb = 0, sb = 0;
    for (int i = 1; i < W.Q; ++i)
        if (mask[g.idx(x - c[i][0], y - c[i][1], z - c[i][2])]) fb |= 1u << i;
    for (int k = 1; k < W.QS; ++k) {
        if (!W.in_x(x - c[k][0])) continue;
        if (mask[g.idx(x - c[k][0], y - c[k][1], z - c[k][2])]) sb |= 1u << k;
    }
    uint32_t w = fb | (sb << W.wet_shift);
    for (int d = 1; d < W.QS; ++d) {
        // neighbour y = n + e_d, reached without crossing a seam, fluid, whose
        // upstream in direction opp(d) (= n + 2 e_d) is solid and in the domain
        if (!W.in_x(x + c[d][0]) || !W.in_x(x + 2 * c[d][0])) continue;
        if (mask[g.idx(x + c[d][0], y + c[d][1], z + c[d][2])]) continue;
        if (mask[g.idx(x + 2 * c[d][0], y + 2 * c[d][1], z + 2 * c[d][2])]) w |= 1u << (W.hop_shift + d);
    }
    if (fb_out) *fb_out = fb;
    if (sb_out) *sb_out = sb;
    return w;
}

}  // namespace

void link_words(const GeomSpec& s, const std::vector<uint8_t>& mask, std::vector<uint32_t>& words,
                std::vector<uint32_t>* flow_bits, std::vector<uint32_t>* solute_bits) {
    const WordCtx W = word_ctx(s);
    const Grid& g = W.g;
    const long long N = (long long)g.nx * g.ny * g.nz;
    words.assign((size_t)N, 0u);
    if (flow_bits) flow_bits->assign((size_t)N, 0u);
    if (solute_bits) solute_bits->assign((size_t)N, 0u);
    parallel_rows(g.ny, g.nz, [&](unsigned, int z, int y) {
        for (int x = 0; x < g.nx; ++x) {
            const long long n = g.idx(x, y, z);
            if (mask[n]) {
                words[n] = 0x80000000u;
                continue;
            }
            uint32_t fb = 0, sb = 0;
            words[n] = word_at(W, mask, x, y, z, &fb, &sb);
            if (flow_bits) (*flow_bits)[n] = fb;
            if (solute_bits) (*solute_bits)[n] = sb;
        }
    });
}

int64_t convert_nodes(const GeomSpec& s, std::vector<uint8_t>& mask, std::vector<unsigned>& pos,
                      std::vector<uint32_t>& words, const std::vector<long long>& add, std::vector<int>& from) {
    const WordCtx W = word_ctx(s);
    const Grid& g = W.g;
    static const int ax[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    // 1. the new solid nodes, then the pinch rule from their axis neighbours
    std::vector<long long> newly, work;
    auto xyz = [&](long long n, int& x, int& y, int& z) {
        x = (int)(n % g.nx);
        y = (int)((n / g.nx) % g.ny);
        z = (int)(n / ((long long)g.nx * g.ny));
    };
    auto push_axis_neighbours = [&](long long n) {
        int x, y, z;
        xyz(n, x, y, z);
        for (int a = 0; a < g.dim; ++a)
            for (int sgn = -1; sgn <= 1; sgn += 2) {
                const int xx = x + sgn * ax[a][0];
                if (g.seam && (xx < 0 || xx >= g.nx)) continue;
                work.push_back(g.idx(xx, y + sgn * ax[a][1], z + sgn * ax[a][2]));
            }
    };
    for (long long n : add)
        if (!mask[n]) {
            mask[n] = 1;
            newly.push_back(n);
            push_axis_neighbours(n);
        }
    while (!work.empty()) {
        const long long n = work.back();
        work.pop_back();
        if (mask[n]) continue;
        int x, y, z;
        xyz(n, x, y, z);
        if (!pinched(g, mask, x, y, z)) continue;
        mask[n] = 1;
        newly.push_back(n);
        push_axis_neighbours(n);
    }
    // 2. the fluid list without them, in the same (band) order
    const long long nf_old = (long long)pos.size();
    std::vector<unsigned> pos_new;
    std::vector<uint32_t> words_new;
    pos_new.reserve((size_t)nf_old);
    words_new.reserve((size_t)nf_old);
    from.clear();
    for (long long k = 0; k < nf_old; ++k) {
        if (mask[pos[k]]) continue;
        pos_new.push_back(pos[k]);
        words_new.push_back(words[k]);
        from.push_back((int)k);
    }
    // 3. link words of the fluid nodes within two nodes of a new solid node
    //    (flow and wet bits look one node upstream, the wet-neighbour bits two)
    std::vector<long long> touched;
    for (long long n : newly) {
        int x, y, z;
        xyz(n, x, y, z);
        for (int dz = (g.dim == 3 ? -2 : 0); dz <= (g.dim == 3 ? 2 : 0); ++dz)
            for (int dy = -2; dy <= 2; ++dy)
                for (int dx = -2; dx <= 2; ++dx) {
                    const long long m = g.idx(x + dx, y + dy, z + dz);
                    if (!mask[m]) touched.push_back(m);
                }
    }
    if (!touched.empty()) {
        std::sort(touched.begin(), touched.end());
        touched.erase(std::unique(touched.begin(), touched.end()), touched.end());
        // new fluid index of each touched node: binary search in the band order
        // is not possible (pos is not sorted by box index), so map them once
        std::vector<int> knew((size_t)g.nx * g.ny * g.nz, -1);
        for (size_t k = 0; k < pos_new.size(); ++k) knew[pos_new[k]] = (int)k;
        for (long long m : touched) {
            int x, y, z;
            xyz(m, x, y, z);
            words_new[(size_t)knew[m]] = word_at(W, mask, x, y, z, nullptr, nullptr);
        }
    }
    pos.swap(pos_new);
    words.swap(words_new);
    return (int64_t)newly.size();
}

}  // namespace mclbm

namespace mclbm {

// Conjugate heat transfer node lists (periodic wrap in every direction):
//   solid list: solid nodes and interface nodes (fluid nodes with a solid
//   flow-lattice neighbour), in the band order of the fluid numbering, the
//   interface nodes of each plane of a band ahead of its solid nodes (so the
//   interface solve, one thread per interface node, reads and writes
//   consecutive solid-list entries);
//   interface list: box index of every interface node (same order) and the
//   bits i of its unknown solid populations: those whose upstream node
//   n - c_i is a fluid node that is not an interface node (nothing streams
//   them), or a fluid node while n + c_i is solid (the solid field does not
//   pass through the fluid).
void thermal_lists(const GeomSpec& s, const std::vector<uint8_t>& mask, int band_rows, std::vector<unsigned>& spos,
                   std::vector<int>& smap, std::vector<unsigned>& iface_box, std::vector<uint32_t>& ms_bits) {
    const int Q = s.lattice == 1 ? 19 : 9;
    const int (*c)[3] = s.lattice == 1 ? C19 : C9;
    const long long N = (long long)s.nx * s.ny * s.nz;
    auto wrap = [](int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); };
    auto at = [&](int x, int y, int z) { return (long long)x + (long long)s.nx * (y + (long long)s.ny * z); };
    std::vector<uint8_t> itf((size_t)N, 0);
    for (int z = 0; z < s.nz; ++z)
        for (int y = 0; y < s.ny; ++y)
            for (int x = 0; x < s.nx; ++x) {
                const long long n = at(x, y, z);
                if (mask[(size_t)n]) continue;
                for (int i = 1; i < Q; ++i)
                    if (mask[(size_t)at(wrap(x - c[i][0], s.nx), wrap(y - c[i][1], s.ny), wrap(z - c[i][2], s.nz))]) {
                        itf[(size_t)n] = 1;
                        break;
                    }
            }
    smap.assign((size_t)N, -1);
    spos.clear();
    iface_box.clear();
    ms_bits.clear();
    for (int y0 = 0; y0 < s.ny; y0 += band_rows)
        for (int z = 0; z < s.nz; ++z)
            for (int pass = 0; pass < 2; ++pass)   // interface nodes, then solid nodes
                for (int y = y0; y < std::min(s.ny, y0 + band_rows); ++y)
                    for (int x = 0; x < s.nx; ++x) {
                        const long long n = at(x, y, z);
                        if (!(pass == 0 ? itf[(size_t)n] : mask[(size_t)n])) continue;
                        smap[(size_t)n] = (int)spos.size();
                        spos.push_back((unsigned)n);
                    }
    for (int y0 = 0; y0 < s.ny; y0 += band_rows)
        for (int z = 0; z < s.nz; ++z)
            for (int y = y0; y < std::min(s.ny, y0 + band_rows); ++y)
                for (int x = 0; x < s.nx; ++x) {
                    const long long n = at(x, y, z);
                    if (!itf[(size_t)n]) continue;
                    uint32_t b = 0;
                    for (int i = 1; i < Q; ++i) {
                        const long long m = at(wrap(x - c[i][0], s.nx), wrap(y - c[i][1], s.ny), wrap(z - c[i][2], s.nz));
                        const long long d = at(wrap(x + c[i][0], s.nx), wrap(y + c[i][1], s.ny), wrap(z + c[i][2], s.nz));
                        // nothing streams it (upstream pure fluid), or it would stream in from
                        // a fluid node across this node from a solid one
                        if (!mask[(size_t)m] && (!itf[(size_t)m] || mask[(size_t)d])) b |= 1u << i;
                    }
                    iface_box.push_back((unsigned)n);
                    ms_bits.push_back(b);
                }
}

}  // namespace mclbm
