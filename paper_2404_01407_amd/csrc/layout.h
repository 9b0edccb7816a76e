// Host-side mesh ingest: validation, colour ordering, colour-major internal numbering
// with locality ordering inside each colour, and the sliced-ELL (SELL-64) layout the
// device kernels stream.  Pure C++ (no HIP): unit-testable without a GPU.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fnlh.h"

namespace fnlh {

constexpr int kTile = 64;  // rows per tile == wavefront width on CDNA

struct Layout {
  int64_t N = 0, E = 0, B = 0;
  int32_t n_zones = 1;
  int32_t n_colours = 0;
  bool bipartite = false;
  std::vector<int32_t> colour_user;  // [N] colour of each user cell
  int64_t NP = 0;                    // internal rows incl. padding (each colour padded to 64)
  std::vector<int32_t> perm;         // [N] user id -> internal row
  std::vector<int32_t> iperm;        // [NP] internal row -> user id, -1 for padding rows
  std::vector<int64_t> cstart;       // [n_colours+1] internal row range of each colour (64-aligned)
  std::vector<int64_t> ccount;       // [n_colours] cells of each colour
  std::vector<int64_t> ctile;        // [n_colours+1] tile range of each colour
  // per colour, for the algorithmic-traffic model of the sweep kernels
  std::vector<int64_t> c_deg;        // couplings leaving rows of the colour
  std::vector<int64_t> c_deg_upper;  // ... to higher colours
  std::vector<int64_t> c_nbr;        // distinct neighbour cells of its rows
  std::vector<int64_t> c_nbr_lower;  // ... of lower colours
  std::vector<int64_t> c_nbr_upper;  // ... of higher colours

  // tile t = internal rows [64t, 64t+64), never straddling a colour
  int64_t n_tiles = 0;
  int64_t n_slots = 0;               // sum of tile widths
  std::vector<int32_t> tile_nrows;   // valid (non-padding) rows, a prefix of the tile
  std::vector<int32_t> tile_width;   // max degree in the tile
  std::vector<int64_t> tile_slot0;   // first slot

  // entries, flat index (slot * 64 + lane)
  std::vector<int32_t> ent_nbr;      // internal neighbour row (padding: the row itself)
  std::vector<int32_t> ent_edge;     // +(e+1) if the row is edge e's first cell, -(e+1) if second, 0 pad
  std::vector<int32_t> ent_rev;      // flat index of the transposed coupling, -1 pad
  std::vector<int64_t> edge_ent;     // [2E] flat entry of coupling (a->b) at 2e, (b->a) at 2e+1

  // per internal row (padding rows: volume 1, zone 0, no faces)
  std::vector<double> vol;           // [NP]
  std::vector<int32_t> zone;         // [NP]
  std::vector<int32_t> bf_ptr;       // [NP+1] boundary faces of each internal row
  std::vector<int32_t> bf_idx;       // [B]  boundary face ids
};

// Validate and build.  Returns FNLH_OK or a negative code with a message in err.
int build_layout(const fnlh_mesh& m, const fnlh_options& o, Layout& L, std::string& err);

// Partition-local ILU(0) in the natural order (section "Parallel Implementation": each
// partition factors and solves its own block of the LHS, the couplings to other
// partitions ignored).  Inside a partition the order is the user cell numbering; a
// cell's level is one more than the highest level among its in-partition neighbours of
// lower number (0 if none), so the cells of one level are never coupled and can be
// processed together.  Consecutive partitions (by ascending label) are grouped into
// work units of at most unit_rows cells (a partition larger than that is a unit of its
// own); a unit is processed by one workgroup, level by level, its partitions' levels
// merged (cells of different partitions are never coupled either).  Positions number
// the cells unit by unit, inside a unit by (level, partition, cell id); the
// in-partition couplings of a position are packed in SELL-64 form over groups of 64
// consecutive positions, lower neighbours first.
struct PiluLayout {
  int64_t n_parts = 0, n_units = 0, n_groups = 0, n_slots = 0;
  int32_t max_part = 0, max_rows = 0, max_levels = 0;  // largest partition, largest unit
  int64_t n_coup = 0;                // in-partition couplings (directed)
  std::vector<int32_t> unit_ptr;     // [n_units+1] position range of each unit
  std::vector<int32_t> unit_lev;     // [n_units+1] level range of each unit (into lev_ptr)
  std::vector<int32_t> lev_ptr;      // [levels+1] position range of each level
  std::vector<int32_t> pos_row;      // [n_groups*64] internal row of each position, -1 past N
  std::vector<int32_t> g_width;      // [n_groups] couplings of the group's widest position
  std::vector<int64_t> g_slot0;      // [n_groups] first packed slot
  std::vector<int32_t> e_pos;        // [n_slots*64] neighbour position, -1 padding
  std::vector<int32_t> e_row;        // [n_slots*64] neighbour internal row, -1 padding
  std::vector<int32_t> e_src;        // [n_slots*64] the coupling's flat entry in the SELL layout
  std::vector<int32_t> e_rev;        // [n_slots*64] packed entry of the transposed coupling
};

// part: [N] partition label of each user cell; unit_rows: cells per work unit (>= 1).
int build_pilu(const Layout& L, const std::vector<int32_t>& part, int32_t unit_rows, PiluLayout& P,
               std::string& err);

}  // namespace fnlh
