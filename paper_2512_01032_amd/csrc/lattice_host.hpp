// lattice_host.hpp -- host-side construction of one lattice's device state:
// parameter validation, node classification, tile table, arena layout and the
// descriptor.  Shared by the single-lattice API and the serving scheduler.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "pflbm.hpp"

namespace pflbm {

void set_error(const char* fmt, ...);

struct LatticeLayout {
    int tx = 64, ty = 4, tz = 16;
    int64_t N = 0;
    int64_t n_fluid = 0, n_ghost = 0, n_solid = 0;
    int64_t n_wall = 0;           // near-wall fluid nodes (each has a slot)
    size_t off_desc = 0, off_counter = 0, off_pop0 = 0, off_pop1 = 0, pop_bytes = 0, off_phi = 0, off_flag = 0,
           off_link = 0, off_tiles = 0, off_partials = 0, off_gbuf = 0, off_ghosts = 0,
           off_wslot = 0, off_hyst = 0, off_wall = 0, off_wgl = 0, off_wrefs = 0, off_wmat = 0,
           total = 0;
    int64_t gface_base[6] = {0, 0, 0, 0, 0, 0};
    int64_t gface_count = 0;      // face-buffer entries (per velocity component)
    std::vector<uint8_t> flag;
    std::vector<uint32_t> link;
    std::vector<int32_t> wslot;   // slot of each near-wall fluid node (-1: none)
    std::vector<double> wall;     // sub-voxel walls: [WALL_ROWS][n_wall] link fractions, normal
    std::vector<Tile> tiles;
    std::vector<GhostRef> ghosts;
    std::vector<WallRef> walls;   // near-wall fluid nodes in slot order (lattice 0)
    std::vector<uint32_t> wmat;   // [3][n_wall]: material of the solid neighbour of link
                                  // i in bits 4 ((i - 1) % 6) of word (i - 1) / 6
};

// Validate parameters (and geometry when given).  Returns LBM_OK or sets the
// error message and returns LBM_E_INVAL.
int validate_params(const lbm_params* p, const lbm_geometry* geo);

// Tile width for a lattice of width nx; tile depth for a given tile count target.
int choose_tx(int nx);
int choose_tz(const lbm_params* p, int tx);
void xcd_order(std::vector<Tile>& t);   // XCD-aware launch order of a tile list

// Size of the phase-field lattice (7 or 19).
inline int phase_q(const lbm_params* p) { return p->q_phase == 19 ? 19 : 7; }

// Bytes per stored population of each lattice.
void storage_sizes(int storage, int* sh, int* sg, int* sphi);

// Sizes only (no geometry): used by lbm_footprint; assumes every tile is kept.
size_t footprint_bytes(const lbm_params* p);

// Full classification + tile table + offsets.  lat: lattice index stamped in
// the tiles.  Returns LBM_OK or LBM_E_INVAL.
int build_layout(const lbm_params* p, const lbm_geometry* geo, int lat, LatticeLayout* L);

// Descriptor for device pointers rooted at base (device address of the arena).
void fill_desc(const lbm_params* p, const lbm_geometry* geo, const LatticeLayout& L,
               char* base, int64_t step, Desc* d);

// Upload flags, links, tiles and descriptor to a device arena at base, then
// initialise the populations (FIELDS or POPULATIONS).  Synchronous on s.
int upload_and_init(const lbm_params* p, const lbm_geometry* geo, const lbm_init* init,
                    LatticeLayout& L, char* base, Desc* hdesc, hipStream_t s);

// Read fields of one lattice whose descriptor is at d_desc and tiles at
// d_tiles (device).  Synchronous.
// parity: AA parity of the lattice's current step.
int read_lattice(int storage, const Desc& hdesc, int parity, Desc* d_desc, const Tile* d_tiles,
                 int ntiles, const WallRef* d_walls, int nwalls, uint32_t mask, double* phi,
                 double* P, double* u, double* pops, hipStream_t s);

// Doubles of device staging read_lattice_staged needs for a mask (every
// population row counts once pops is given with LBM_POP_H or LBM_POP_G).
size_t read_staging_elems(const Desc& hdesc, uint32_t mask, const double* phi, const double* P,
                          const double* u, const double* pops);
// read_lattice with caller-provided device staging buf of at least
// read_staging_elems() doubles: allocates nothing.  Synchronous.
int read_lattice_staged(int storage, const Desc& hdesc, int parity, Desc* d_desc, const Tile* d_tiles,
                        int ntiles, const WallRef* d_walls, int nwalls, uint32_t mask, double* phi,
                        double* P, double* u, double* pops, double* buf, hipStream_t s);

}  // namespace pflbm
