// Host-side geometry preparation (pinch-fill, link words).
#pragma once

#include <stdint.h>

#include <vector>

namespace mclbm {

struct GeomSpec {
    int lattice;  // 0 D2Q9/D2Q5, 1 D3Q19/D3Q7
    int nx, ny, nz;
    int solute;   // 2 = inlet/outlet seams in x
};

// Reclassify pinched fluid voxels as solid (in place); returns their count.
int64_t pinch_fill(const GeomSpec& s, std::vector<uint8_t>& mask);

// Build the per-node link words used by the kernels (bit layout in
// common.hpp) and, optionally, the plain flow / wet-link bit masks.
void link_words(const GeomSpec& s, const std::vector<uint8_t>& mask, std::vector<uint32_t>& words,
                std::vector<uint32_t>* flow_bits, std::vector<uint32_t>* solute_bits);

// Turns the fluid nodes listed in `add` (box indices) solid, applies the pinch
// rule from them, and updates in place: mask, pos (fluid index -> box index, in
// the same band order without the nodes that turned solid) and words (link
// word of each fluid node, recomputed where a new solid node is within two
// nodes).  from[k] receives the old fluid index of new fluid node k.  Returns
// the number of nodes that turned solid.  The result equals pinch_fill and
// link_words applied to the new mask.
int64_t convert_nodes(const GeomSpec& s, std::vector<uint8_t>& mask, std::vector<unsigned>& pos,
                      std::vector<uint32_t>& words, const std::vector<long long>& add, std::vector<int>& from);

// Conjugate heat transfer: solid list (solid and interface nodes, band order
// with band_rows rows per band; spos = box index, smap = box -> list index or
// -1), interface nodes (box indices, same order) and, per interface node, the
// bits i of its unknown solid populations (upstream n - c_i a fluid node that
// is not an interface node, or a fluid node while n + c_i is solid).
void thermal_lists(const GeomSpec& s, const std::vector<uint8_t>& mask, int band_rows, std::vector<unsigned>& spos,
                   std::vector<int>& smap, std::vector<unsigned>& iface_box, std::vector<uint32_t>& ms_bits);

}  // namespace mclbm
