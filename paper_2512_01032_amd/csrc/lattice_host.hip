// lattice_host.hip -- validation, classification, tile table and
// initialisation of one lattice (see lattice_host.hpp).
#include "lattice_host.hpp"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>

namespace pflbm {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

}  // namespace pflbm

extern "C" const char* lbm_last_error(void) { return pflbm::g_err; }

namespace pflbm {

static const int HCX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int HCY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int HCZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
static double host_wg(int i) { return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

void storage_sizes(int storage, int* sh, int* sg, int* sphi) {
    switch (storage) {
        case ST_FP64: *sh = 8; *sg = 8; *sphi = 8; break;
        case ST_FP32:
        case ST_FP32_SHIFT: *sh = 4; *sg = 4; *sphi = 4; break;
        case ST_FP16_G: *sh = 4; *sg = 2; *sphi = 4; break;
        default: *sh = 2; *sg = 2; *sphi = 4; break;
    }
}

// bytes of one population group (pop_layout): nodes of the row-padded
// lattice times the group's bytes per node
int64_t pop_group_bytes(const lbm_params* p) {
    int sh, sg, sphi;
    storage_sizes(p->storage, &sh, &sg, &sphi);
    const PopLayout pl = pop_layout(phase_q(p), sh, sg);
    return (int64_t)pad_row(p->nx) * p->ny * p->nz * pl.pb;
}

int validate_params(const lbm_params* p, const lbm_geometry* geo) {
    if (!p) { set_error("params is NULL"); return LBM_E_INVAL; }
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) {
        set_error("lattice size %d x %d x %d: every dimension must be >= 1", p->nx, p->ny, p->nz);
        return LBM_E_INVAL;
    }
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    if (N >= ((int64_t)1 << 31)) { set_error("lattice of %lld nodes exceeds 2^31", (long long)N); return LBM_E_INVAL; }
    if (p->storage < ST_FP64 || p->storage > ST_FP16_ALL) { set_error("unknown storage mode %d", p->storage); return LBM_E_INVAL; }
    if (p->storage == ST_FP16_ALL) {
        // 11 significant bits on the h deviations leave phi = sum h_i with
        // rounding noise of ~1e-4 per step, which the counter-term of Eqs. 2-4
        // and the switches of Eq. 5 amplify to phi errors of ~1e-1: no stated
        // bound holds, so the mode is not offered
        set_error("storage LBM_FP16_SHIFT_ALL is not supported: FP16 phase-field populations "
                  "give no bounded phi error; use LBM_FP16_SHIFT_G");
        return LBM_E_INVAL;
    }
    if (p->q_phase != 0 && p->q_phase != 7 && p->q_phase != 19) {
        set_error("q_phase %d: the phase lattice is D3Q7 (7) or D3Q19 (19)", p->q_phase);
        return LBM_E_INVAL;
    }
    {
        // every population group is one buffer resource of at most 4 GiB
        const int64_t big = pop_group_bytes(p);
        if (big >= ((int64_t)1 << 32)) {
            set_error("lattice of %lld nodes (rows padded to %d): a population group of %lld bytes exceeds "
                      "4 GiB in this storage mode", (long long)N, pad_row(p->nx), (long long)big);
            return LBM_E_INVAL;
        }
    }
    if (p->subvoxel != 0 && p->subvoxel != 1) {
        set_error("subvoxel %d: 0 (voxel walls) or 1 (walls from a signed distance)", p->subvoxel);
        return LBM_E_INVAL;
    }
    if (geo && (p->subvoxel != 0) != (geo->sdf != nullptr)) {
        set_error(p->subvoxel ? "subvoxel = 1 needs geometry.sdf" : "geometry.sdf is given but subvoxel = 0");
        return LBM_E_INVAL;
    }
    if (p->hysteresis < 0 || p->hysteresis > 2) {
        set_error("hysteresis %d: 0 (off), 1 or 2", p->hysteresis);
        return LBM_E_INVAL;
    }
    if (p->hysteresis && !(p->hyst_beta >= 0.0 && p->hyst_beta < 1.0)) {
        set_error("hyst_beta %g outside [0, 1)", p->hyst_beta);
        return LBM_E_INVAL;
    }
    if (!(p->rho_l > 0) || !(p->rho_g > 0)) { set_error("densities must be > 0"); return LBM_E_INVAL; }
    if (!(p->nu_l > 0) || !(p->nu_g > 0)) { set_error("viscosities must be > 0 (tau > 1/2)"); return LBM_E_INVAL; }
    if (!(p->W > 0)) { set_error("interface width W must be > 0"); return LBM_E_INVAL; }
    if (!(p->M > 0)) { set_error("mobility M must be > 0"); return LBM_E_INVAL; }
    if (!(p->sigma >= 0)) { set_error("surface tension must be >= 0"); return LBM_E_INVAL; }
    if (!(p->eps > 0)) { set_error("eps must be > 0"); return LBM_E_INVAL; }
    if (p->mobility_corr && !(p->mc_D > 0)) { set_error("mobility correction needs D > 0"); return LBM_E_INVAL; }
    if (p->mix == LBM_MIX_TANH && !(p->mix_width > 0)) { set_error("mix_width must be > 0"); return LBM_E_INVAL; }
    if (p->mix != LBM_MIX_LINEAR && p->mix != LBM_MIX_TANH) { set_error("unknown mix %d", p->mix); return LBM_E_INVAL; }
    if (p->friction != LBM_FRICTION_NOSLIP && p->friction != LBM_FRICTION_INTERFACE_SLIP &&
        p->friction != LBM_FRICTION_PARTIAL_SLIP) {
        set_error("unknown friction %d", p->friction); return LBM_E_INVAL;
    }
    if (p->friction == LBM_FRICTION_PARTIAL_SLIP && !(p->slip_factor >= 0.0 && p->slip_factor <= 1.0)) {
        set_error("slip_factor %g outside [0, 1]", p->slip_factor); return LBM_E_INVAL;
    }
    const int dims[3] = {p->nx, p->ny, p->nz};
    for (int f = 0; f < 6; ++f) {
        if (p->face_bc[f] != LBM_BC_PERIODIC && p->face_bc[f] != LBM_BC_PRESSURE) {
            set_error("face %d: unknown boundary type %d", f, p->face_bc[f]); return LBM_E_INVAL;
        }
        if (p->face_bc[f] == LBM_BC_PRESSURE && dims[f / 2] < 3) {
            set_error("face %d: a pressure face needs >= 3 nodes along its axis", f); return LBM_E_INVAL;
        }
    }
    if (geo) {
        for (int k = 0; k < 16; ++k)
            if (!(geo->theta_deg[k] > 0.0 && geo->theta_deg[k] < 180.0)) {
                set_error("contact angle of material %d must lie in (0, 180) degrees", k);
                return LBM_E_INVAL;
            }
    }
    return LBM_OK;
}

int choose_tx(int nx) {
    // fewest idle lanes on the ragged x end; among equals the widest tile
    int best = 64, waste_best = 1 << 30;
    for (int tx : {64, 32, 16}) {
        const int waste = ((nx + tx - 1) / tx) * tx - nx;
        if (waste < waste_best) { waste_best = waste; best = tx; }
    }
    return best;
}

int choose_tz(const lbm_params* p, int tx) {
    const char* env = getenv("LBM_TILE_Z");
    if (env && atoi(env) > 0) return std::min(atoi(env), p->nz);
    const int ty = NTHREADS / tx;
    const int64_t cols = (int64_t)((p->nx + tx - 1) / tx) * ((p->ny + ty - 1) / ty);
    // Short z-chunks: a tile's set-up (three staged phi planes) is cheap, and
    // many more tiles than resident blocks (4 per CU x 256 CUs) leave no
    // half-empty last round.  2 planes with 4- and 8-byte g populations, 4
    // with 2-byte ones, whose cheaper planes amortise the set-up over more
    // (256 x 256 x 512 duct: FP32 18.35 / 18.72 / 18.86 G fluid updates/s
    // at 8 / 4 / 2 planes, FP16 g 25.33 / 25.33 / 24.47, FP64 9.42 / 9.52 /
    // 9.54); halved down to 2 until the lattice has >= 4096 tiles.
    int sh, sg, sphi;
    storage_sizes(p->storage, &sh, &sg, &sphi);
    int tz = sg == 2 ? 4 : 2;
    while (tz > 2 && cols * ((p->nz + tz - 1) / tz) < 4096) tz /= 2;
    return std::min(tz, p->nz);
}

// Workgroups go to the eight XCDs round-robin (block b to XCD b mod 8), and
// each XCD has its own L2.  The tile list (x fastest, then y, then z) is cut
// into eight contiguous segments and interleaved so that XCD k walks segment
// k in order: tiles that share cache lines (the x-neighbours of a row, whose
// odd-step accesses straddle the row's tile edges, and the phi halo rows)
// meet in one L2.  Segment lengths differ by at most one; the longer ones
// come first, so only the final round has fewer than eight blocks.
void xcd_order(std::vector<Tile>& t) {
    constexpr int NX = 8;
    const int64_t n = (int64_t)t.size();
    const char* env = getenv("LBM_TILE_ORDER");
    if (n < 2 * NX || (env && strcmp(env, "spatial") == 0)) return;
    const int64_t S = (n + NX - 1) / NX, r = n - NX * (S - 1);
    std::vector<Tile> o;
    o.reserve((size_t)n);
    for (int64_t j = 0; j < S; ++j)
        for (int64_t k = 0; k < NX; ++k) {
            const int64_t len = S - 1 + (k < r ? 1 : 0), start = k * (S - 1) + std::min<int64_t>(k, r);
            if (j < len) o.push_back(t[(size_t)(start + j)]);
        }
    t.swap(o);
}

static void face_planes(const lbm_params* p, LatticeLayout* L) {
    int64_t b = 0;
    for (int f = 0; f < 6; ++f) {
        L->gface_base[f] = b;
        if (p->face_bc[f] != LBM_BC_PRESSURE) continue;
        const int ax = f / 2;
        b += ax == 0 ? (int64_t)p->ny * p->nz : (ax == 1 ? (int64_t)p->nx * p->nz
                                                         : (int64_t)p->nx * p->ny);
    }
    L->gface_count = b;
}

static void layout_offsets(const lbm_params* p, int64_t ntiles, int64_t nghosts,
                           LatticeLayout* L) {
    int sh, sg, sphi;
    storage_sizes(p->storage, &sh, &sg, &sphi);
    const int64_t N = L->N;
    face_planes(p, L);
    size_t o = 0;
    L->off_desc = o; o = align256(o + sizeof(Desc));
    L->off_counter = o; o = align256(o + sizeof(unsigned int));
    {
        const PopLayout pl = pop_layout(phase_q(p), sh, sg);
        L->pop_bytes = (size_t)pop_group_bytes(p);
        L->off_pop0 = o; o = align256(o + L->pop_bytes);
        L->off_pop1 = L->off_pop0;
        if (pl.G == 2) { L->off_pop1 = o; o = align256(o + L->pop_bytes); }
    }
    L->off_phi = o; o = align256(o + (size_t)N * sphi);
    L->off_flag = o; o = align256(o + (size_t)N);
    L->off_link = o; o = align256(o + (size_t)N * 4);
    L->off_tiles = o; o = align256(o + (size_t)ntiles * sizeof(Tile));
    L->off_partials = o; o = align256(o + (size_t)ntiles * NPART * sizeof(double));
    L->off_gbuf = o; o = align256(o + (size_t)3 * L->gface_count * sphi);
    L->off_ghosts = o; o = align256(o + (size_t)nghosts * sizeof(GhostRef));
    // per-node slot of near-wall fluid nodes (hysteresis, sub-voxel walls);
    // hysteresis: 18 wall values per slot; sub-voxel walls: 18 link
    // fractions and the wall normal per slot
    L->off_wslot = o; o = align256(o + (size_t)N * 4);
    L->off_wgl = o; o = align256(o + (size_t)WG_ROWS * L->n_wall * sphi);
    L->off_wrefs = o; o = align256(o + (size_t)L->n_wall * sizeof(WallRef));
    L->off_wmat = o; o = align256(o + (size_t)3 * L->n_wall * 4);
    L->off_hyst = o; if (p->hysteresis) o = align256(o + (size_t)(QG - 1) * L->n_wall * sphi);
    L->off_wall = o; if (p->subvoxel) o = align256(o + (size_t)WALL_ROWS * L->n_wall * sphi);
    L->total = o;
}

size_t footprint_bytes(const lbm_params* p) {
    if (validate_params(p, nullptr) != LBM_OK) return 0;
    LatticeLayout L;
    L.N = (int64_t)p->nx * p->ny * p->nz;
    const int tx = choose_tx(p->nx), ty = NTHREADS / tx, tz = choose_tz(p, tx);
    const int64_t ntiles = (int64_t)((p->nx + tx - 1) / tx) * ((p->ny + ty - 1) / ty) *
                           ((p->nz + tz - 1) / tz);
    face_planes(p, &L);
    L.n_wall = L.N;                                  // bound: every node near a wall
    layout_offsets(p, ntiles, L.gface_count, &L);   // ghosts <= face entries
    return L.total;
}

int build_layout(const lbm_params* p, const lbm_geometry* geo, int lat, LatticeLayout* L) {
    int rc = validate_params(p, geo);
    if (rc != LBM_OK) return rc;
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    const int64_t N = (int64_t)nx * ny * nz;
    L->N = N;
    L->flag.assign(N, 0);
    L->link.assign(N, 0);
    const uint8_t* solid = geo ? geo->solid : nullptr;
    auto idx = [&](int x, int y, int z) -> int64_t {
        x = ((x % nx) + nx) % nx; y = ((y % ny) + ny) % ny; z = ((z % nz) + nz) % nz;
        return x + (int64_t)nx * (y + (int64_t)ny * z);
    };
    int64_t nf = 0, ng = 0, ns = 0;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int64_t n = x + (int64_t)nx * (y + (int64_t)ny * z);
                if (solid && solid[n]) {
                    if (solid[n] > 16) { set_error("node %lld: material id %d > 16", (long long)n, solid[n]); return LBM_E_INVAL; }
                    L->flag[n] = make_flag(KIND_SOLID, solid[n] - 1);
                    ++ns;
                    continue;
                }
                const int c[3] = {x, y, z}, d[3] = {nx, ny, nz};
                int face = -1, count = 0;
                for (int f = 0; f < 6; ++f) {
                    if (p->face_bc[f] != LBM_BC_PRESSURE) continue;
                    const int layer = (f & 1) ? d[f / 2] - 1 : 0;
                    if (c[f / 2] == layer) { face = f; ++count; }
                }
                if (count > 1) {
                    set_error("node (%d,%d,%d) lies on two pressure faces; make it solid", x, y, z);
                    return LBM_E_INVAL;
                }
                if (count == 1) { L->flag[n] = make_flag(KIND_GHOST, face); ++ng; }
                else { L->flag[n] = make_flag(KIND_FLUID, 0); ++nf; }
            }
    L->n_fluid = nf; L->n_ghost = ng; L->n_solid = ns;
    if (nf == 0) { set_error("the lattice has no fluid node"); return LBM_E_INVAL; }
    // ghost owners
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int64_t n = x + (int64_t)nx * (y + (int64_t)ny * z);
                if (flag_kind(L->flag[n]) != KIND_GHOST) continue;
                const int face = flag_sub(L->flag[n]);
                const int ax = face / 2, sg = (face & 1) ? -1 : 1;
                const int64_t o = idx(x + (ax == 0 ? sg : 0), y + (ax == 1 ? sg : 0), z + (ax == 2 ? sg : 0));
                if (flag_kind(L->flag[o]) != KIND_FLUID) {
                    set_error("pressure ghost (%d,%d,%d): its inward neighbour must be fluid", x, y, z);
                    return LBM_E_INVAL;
                }
                L->ghosts.push_back(GhostRef{lat, (int32_t)n});
                L->flag[o] |= F_OWNER;
                L->link[o] |= 1u << (LINK_OWNER_SHIFT + face);
            }
    // solid links of fluid nodes
    for (int z = 0; z < nz; ++z) {
        const int64_t Z[3] = {(int64_t)((z + nz - 1) % nz) * nx * ny, (int64_t)z * nx * ny,
                              (int64_t)((z + 1) % nz) * nx * ny};
        for (int y = 0; y < ny; ++y) {
            const int64_t Y[3] = {(int64_t)((y + ny - 1) % ny) * nx, (int64_t)y * nx,
                                  (int64_t)((y + 1) % ny) * nx};
            for (int x = 0; x < nx; ++x) {
                const int64_t n = x + Y[1] + Z[1];
                if (flag_kind(L->flag[n]) != KIND_FLUID) continue;
                const int64_t X[3] = {(x + nx - 1) % nx, x, (x + 1) % nx};
                uint32_t m = 0;
                for (int i = 1; i < 19; ++i)
                    if (flag_kind(L->flag[X[HCX[i] + 1] + Y[HCY[i] + 1] + Z[HCZ[i] + 1]]) == KIND_SOLID)
                        m |= 1u << i;
                if (m) { L->link[n] |= m; L->flag[n] |= F_NEAR_WALL; }
            }
        }
    }
    // slots of the near-wall fluid nodes, in node order (coalesced along x)
    L->n_wall = 0;
    std::vector<double>().swap(L->wall);
    L->wslot.assign(N, -1);
    L->walls.clear();
    for (int64_t n = 0; n < N; ++n)
        if ((L->link[n] & SOLID_MASK) && flag_kind(L->flag[n]) == KIND_FLUID) {
            L->walls.push_back(WallRef{0, (int32_t)n, (int32_t)L->n_wall, L->link[n] & SOLID_MASK});
            L->wslot[n] = (int32_t)L->n_wall++;
        }
    // materials of the solid links, packed per slot
    L->wmat.assign((size_t)3 * L->n_wall, 0u);
    for (const WallRef& w : L->walls) {
        const int64_t n = w.node;
        const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
        for (int i = 1; i < 19; ++i) {
            if (!((L->link[n] >> i) & 1u)) continue;
            const int64_t m = (x + HCX[i] + nx) % nx + (int64_t)nx * ((y + HCY[i] + ny) % ny + (int64_t)ny * ((z + HCZ[i] + nz) % nz));
            L->wmat[(size_t)((i - 1) / 6) * L->n_wall + w.slot] |= (uint32_t)flag_sub(L->flag[m]) << (4 * ((i - 1) % 6));
        }
    }
    if (p->subvoxel) {
        // sub-voxel walls from the signed distance (> 0 in the fluid): the
        // link from fluid node x to solid node x + c_i crosses the surface at
        // q = sdf(x) / (sdf(x) - sdf(x + c_i)); the wall normal is the
        // normalised central-difference gradient of sdf (D3Q19 weights), or
        // the solid-link rule where that gradient vanishes
        const double* sdf = geo->sdf;
        const int64_t nw = L->n_wall;
        L->wall.assign((size_t)WALL_ROWS * nw, 0.0);
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    const int64_t n = x + (int64_t)nx * (y + (int64_t)ny * z);
                    const int32_t sl = L->wslot[n];
                    if (sl < 0) continue;
                    const uint32_t m = L->link[n] & SOLID_MASK;
                    double gsd[3] = {0.0, 0.0, 0.0}, vox[3] = {0.0, 0.0, 0.0};
                    for (int i = 1; i < 19; ++i) {
                        const int64_t np = idx(x + HCX[i], y + HCY[i], z + HCZ[i]);
                        const int64_t nm = idx(x - HCX[i], y - HCY[i], z - HCZ[i]);
                        const double d = sdf[np] - sdf[nm];
                        gsd[0] += host_wg(i) * HCX[i] * d;
                        gsd[1] += host_wg(i) * HCY[i] * d;
                        gsd[2] += host_wg(i) * HCZ[i] * d;
                        if (!((m >> i) & 1u)) continue;
                        vox[0] -= host_wg(i) * HCX[i];
                        vox[1] -= host_wg(i) * HCY[i];
                        vox[2] -= host_wg(i) * HCZ[i];
                        const double a = sdf[n], b = sdf[np];
                        if (!(a > 0.0) || !(b <= 0.0)) {
                            set_error("sdf at (%d,%d,%d) = %g and its solid neighbour along link %d = %g "
                                      "do not straddle the wall surface", x, y, z, a, i, b);
                            return LBM_E_INVAL;
                        }
                        L->wall[(size_t)(i - 1) * nw + sl] = a / (a - b);
                    }
                    double gn = sqrt(gsd[0] * gsd[0] + gsd[1] * gsd[1] + gsd[2] * gsd[2]);
                    const double* v = gsd;
                    if (!(gn > 0.0)) {
                        v = vox;
                        gn = sqrt(vox[0] * vox[0] + vox[1] * vox[1] + vox[2] * vox[2]);
                    }
                    for (int a = 0; a < 3; ++a)
                        L->wall[(size_t)(QG - 1 + a) * nw + sl] = gn > 0.0 ? v[a] / gn : 0.0;
                }
    }
    // tile table: keep tiles holding at least one non-solid node
    const int tx = choose_tx(nx), ty = NTHREADS / tx, tz = choose_tz(p, tx);
    L->tx = tx; L->ty = ty; L->tz = tz;
    L->tiles.clear();
    for (int z0 = 0; z0 < nz; z0 += tz)
        for (int y0 = 0; y0 < ny; y0 += ty)
            for (int x0 = 0; x0 < nx; x0 += tx) {
                bool any = false;
                const int z1 = std::min(nz, z0 + tz), y1 = std::min(ny, y0 + ty), x1 = std::min(nx, x0 + tx);
                for (int z = z0; z < z1 && !any; ++z)
                    for (int y = y0; y < y1 && !any; ++y)
                        for (int x = x0; x < x1; ++x)
                            if (flag_kind(L->flag[x + (int64_t)nx * (y + (int64_t)ny * z)]) != KIND_SOLID) { any = true; break; }
                if (!any) continue;
                Tile t;
                memset(&t, 0, sizeof(t));
                t.lat = lat; t.x0 = x0; t.y0 = y0; t.z0 = z0; t.zn = z1 - z0;
                L->tiles.push_back(t);
            }
    xcd_order(L->tiles);
    for (size_t k = 0; k < L->tiles.size(); ++k) L->tiles[k].tile_in_lat = (int)k;
    layout_offsets(p, (int64_t)L->tiles.size(), (int64_t)L->ghosts.size(), L);
    return LBM_OK;
}

void fill_desc(const lbm_params* p, const lbm_geometry* geo, const LatticeLayout& L, char* base,
               int64_t step, Desc* d) {
    memset(d, 0, sizeof(*d));
    d->nx = p->nx; d->ny = p->ny; d->nz = p->nz; d->tx = L.tx;
    d->N = L.N;
    d->storage = p->storage;
    d->ntiles = (int)L.tiles.size();
    d->nxp = pad_row(p->nx);
    d->Np = (int64_t)d->nxp * p->ny * p->nz;
    d->pops[0] = base + L.off_pop0;
    d->pops[1] = base + L.off_pop1;
    d->phi = base + L.off_phi;
    d->flag = (const uint8_t*)(base + L.off_flag);
    d->link = (const uint32_t*)(base + L.off_link);
    d->partials = (double*)(base + L.off_partials);
    d->gbuf = base + L.off_gbuf;
    d->q_phase = phase_q(p);
    d->hysteresis = p->hysteresis;
    d->hyst_reset = 0;
    d->n_wall = L.n_wall;
    d->wslot = (const int32_t*)(base + L.off_wslot);
    d->wgl = base + L.off_wgl;
    d->wmat = (const uint32_t*)(base + L.off_wmat);
    d->hyst = p->hysteresis ? (void*)(base + L.off_hyst) : nullptr;
    d->subvoxel = p->subvoxel ? 1 : 0;
    d->wall = p->subvoxel ? (void*)(base + L.off_wall) : nullptr;
    for (int f = 0; f < 6; ++f) d->gface_base[f] = L.gface_base[f];
    d->gface_count = L.gface_count;
    d->counter = (unsigned int*)(base + L.off_counter);
    d->step = step;
    d->t0 = 0;
    d->stop_step = INT64_MAX;
    d->diag_every = p->diag_every > 0 ? p->diag_every : 0;
    d->rho_l = p->rho_l; d->rho_g = p->rho_g; d->nu_l = p->nu_l; d->nu_g = p->nu_g;
    d->sigma = p->sigma; d->W = p->W; d->M = p->M;
    for (int a = 0; a < 3; ++a) d->F[a] = p->F_ex[a];
    d->mobility_corr = p->mobility_corr ? 1 : 0;
    d->mix = p->mix; d->friction = p->friction;
    d->mc_gamma = p->mc_gamma; d->mc_phi_M = p->mc_phi_M; d->mc_phi_m = p->mc_phi_m;
    d->mc_D = p->mobility_corr ? p->mc_D : 1.0;
    d->eps = p->eps;
    d->mix_phi = p->mix_phi; d->mix_width = p->mix == LBM_MIX_TANH ? p->mix_width : 1.0;
    d->slip_lo = p->slip_lo; d->slip_hi = p->slip_hi;
    d->P_ref = p->P_ref;
    for (int f = 0; f < 6; ++f) {
        d->face_bc[f] = p->face_bc[f];
        d->face_P[f] = p->face_P[f];
        d->face_ramp[f] = p->face_ramp[f];
    }
    for (int k = 0; k < 16; ++k) {
        const double th = geo ? geo->theta_deg[k] * M_PI / 180.0 : M_PI / 2;
        d->cos_t[k] = cos(th);
        d->sin_t[k] = sin(th);
    }
    const bool shifted = p->storage >= ST_FP32_SHIFT;
    d->clamp_a = p->storage == ST_FP64 ? 1e-12 : 1.2e-7;
    d->href = shifted ? 0.5 : 0.0;
    d->gref = shifted ? p->P_ref * 3.0 : 0.0;
    const int ksh = p->fp16_log2_scale_h ? p->fp16_log2_scale_h : 3;
    const int ksg = p->fp16_log2_scale_g ? p->fp16_log2_scale_g : 10;
    (void)ksh;                                   // h is never stored in FP16
    d->scale_h = 1.0;
    d->scale_g = p->storage >= ST_FP16_G ? ldexp(1.0, ksg) : 1.0;
    d->u_max = p->u_max;
    // derived constants (Eq. 4 theta coefficient, Eq. 5 correction factor,
    // Eq. 9 chemical-potential coefficients, Eqs. 10-12 relaxation times)
    const double TG = 1.0 / 3.0, TH = phase_q(p) == 19 ? 1.0 / 3.0 : 0.25;
    double v[PI_COUNT];
    v[PI_RHO_G] = p->rho_g;
    v[PI_RDIF] = p->rho_l - p->rho_g;
    v[PI_MU3] = 48.0 * p->sigma / p->W;
    v[PI_MULAP] = 1.5 * p->sigma * p->W;
    v[PI_TAU_G] = p->nu_g / TG + 0.5;
    v[PI_TAU_L] = p->nu_l / TG + 0.5;
    v[PI_THETA0] = p->M / TH / p->W;
    v[PI_MC_K] = p->mobility_corr ? p->mc_gamma * p->M / (TH * p->W) : 0.0;
    v[PI_MC_INVD] = 1.0 / d->mc_D;
    v[PI_MC_PHI_M] = p->mc_phi_M;
    v[PI_MC_PHI_m] = p->mc_phi_m;
    v[PI_EPS] = p->eps;
    v[PI_MIX_PHI] = p->mix_phi;
    v[PI_MIX_INVW] = 1.0 / d->mix_width;
    v[PI_SLIP_LO] = p->slip_lo;
    v[PI_SLIP_HI] = p->slip_hi;
    v[PI_CLAMP_A] = d->clamp_a;
    v[PI_HREF] = d->href;
    v[PI_GREF] = d->gref;
    v[PI_SH] = d->scale_h;
    v[PI_SG] = d->scale_g;
    v[PI_INV_SH] = 1.0 / d->scale_h;
    v[PI_INV_SG] = 1.0 / d->scale_g;
    v[PI_ITAU_H] = 1.0 / (p->M / TH + 0.5);
    v[PI_FX] = p->F_ex[0];
    v[PI_FY] = p->F_ex[1];
    v[PI_FZ] = p->F_ex[2];
    v[PI_K2W] = 2.0 / p->W;
    v[PI_PREF_DEV] = p->P_ref / TG - d->gref;
    v[PI_HBETA] = p->hysteresis ? p->hyst_beta : 0.0;
    v[PI_HBETA1] = 1.0 - v[PI_HBETA];
    // moving-wall term of the slip band: 2 w_i rho (c_i . u_w) / T_g with
    // u_w = slip_factor * tangential u, as w_i (6 slip_factor rho) (c_i . u_t)
    v[PI_SLIP_W6] = 6.0 * (p->friction == LBM_FRICTION_PARTIAL_SLIP ? p->slip_factor : 1.0);
    for (int k = 0; k < PI_COUNT; ++k) {
        d->pd[k] = v[k];
        d->pf[k] = (float)v[k];
    }
}

#define HIPCHK(expr)                                                              \
    do {                                                                          \
        hipError_t e_ = (expr);                                                   \
        if (e_ != hipSuccess) {                                                   \
            set_error("%s failed: %s", #expr, hipGetErrorString(e_));             \
            return LBM_E_DEVICE;                                                  \
        }                                                                         \
    } while (0)

int upload_and_init(const lbm_params* p, const lbm_geometry* geo, const lbm_init* init,
                    LatticeLayout& L, char* base, Desc* hdesc, hipStream_t s) {
    const int64_t N = L.N;
    int sh, sg, sphi;
    storage_sizes(p->storage, &sh, &sg, &sphi);
    // zero populations and phi (solid slots stay zero), upload geometry
    HIPCHK(hipMemsetAsync(base + L.off_pop0, 0, L.pop_bytes, s));
    if (L.off_pop1 != L.off_pop0) HIPCHK(hipMemsetAsync(base + L.off_pop1, 0, L.pop_bytes, s));
    HIPCHK(hipMemsetAsync(base + L.off_counter, 0, sizeof(unsigned int), s));
    HIPCHK(hipMemsetAsync(base + L.off_partials, 0, L.tiles.size() * NPART * sizeof(double), s));
    HIPCHK(hipMemcpyAsync(base + L.off_flag, L.flag.data(), N, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(base + L.off_link, L.link.data(), (size_t)N * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(base + L.off_wslot, L.wslot.data(), (size_t)N * 4, hipMemcpyHostToDevice, s));
    if (L.n_wall) {
        HIPCHK(hipMemcpyAsync(base + L.off_wrefs, L.walls.data(), L.walls.size() * sizeof(WallRef),
                              hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(base + L.off_wmat, L.wmat.data(), L.wmat.size() * 4, hipMemcpyHostToDevice, s));
    }
    if (p->subvoxel && L.n_wall) {
        // wall table in the compute type (a synchronous copy: the host
        // buffer is temporary)
        const size_t cnt = (size_t)WALL_ROWS * L.n_wall;
        if (sphi == 8) {
            HIPCHK(hipMemcpyAsync(base + L.off_wall, L.wall.data(), cnt * 8, hipMemcpyHostToDevice, s));
            HIPCHK(hipStreamSynchronize(s));
        } else {
            std::vector<float> wf(cnt);
            for (size_t k = 0; k < cnt; ++k) wf[k] = (float)L.wall[k];
            HIPCHK(hipMemcpyAsync(base + L.off_wall, wf.data(), cnt * 4, hipMemcpyHostToDevice, s));
            HIPCHK(hipStreamSynchronize(s));
        }
    }
    HIPCHK(hipMemcpyAsync(base + L.off_tiles, L.tiles.data(), L.tiles.size() * sizeof(Tile),
                          hipMemcpyHostToDevice, s));
    if (!L.ghosts.empty())
        HIPCHK(hipMemcpyAsync(base + L.off_ghosts, L.ghosts.data(), L.ghosts.size() * sizeof(GhostRef),
                              hipMemcpyHostToDevice, s));
    if (L.gface_count)
        HIPCHK(hipMemsetAsync(base + L.off_gbuf, 0, (size_t)3 * L.gface_count * sphi, s));
    const int64_t step0 = (init && init->kind == LBM_INIT_POPULATIONS) ? init->step : 0;
    fill_desc(p, geo, L, base, step0, hdesc);
    HIPCHK(hipMemcpyAsync(base + L.off_desc, hdesc, sizeof(Desc), hipMemcpyHostToDevice, s));
    Desc* ddesc = (Desc*)(base + L.off_desc);
    const Tile* dtiles = (const Tile*)(base + L.off_tiles);
    const int nt = (int)L.tiles.size();
    if (!init) { set_error("init is NULL"); return LBM_E_INVAL; }
    if (init->kind == LBM_INIT_POPULATIONS) {
        if (!init->pops) { set_error("POPULATIONS init needs pops"); return LBM_E_INVAL; }
        double* dpops = nullptr;
        HIPCHK(hipMalloc(&dpops, (size_t)(phase_q(p) + QG) * N * sizeof(double)));
        hipError_t e = hipMemcpyAsync(dpops, init->pops, (size_t)(phase_q(p) + QG) * N * sizeof(double),
                                      hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = launch_restore(p->storage, phase_q(p), (int)(step0 & 1), ddesc, dtiles, nt, dpops, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        hipFree(dpops);
        if (e != hipSuccess) { set_error("restore: %s", hipGetErrorString(e)); return LBM_E_DEVICE; }
        if (p->hysteresis) {
            // the wall-value history restarts from the restored state: a read
            // pass with hyst_reset set records the current wall values
            const int32_t on = 1, off = 0;
            HIPCHK(hipMemcpyAsync(&ddesc->hyst_reset, &on, sizeof(on), hipMemcpyHostToDevice, s));
            HIPCHK(hipStreamSynchronize(s));
            int rc = read_lattice(p->storage, *hdesc, (int)(step0 & 1), ddesc, dtiles, nt,
                                  (const WallRef*)(base + L.off_wrefs), (int)L.n_wall, 0, nullptr,
                                  nullptr, nullptr, nullptr, s);
            HIPCHK(hipMemcpyAsync(&ddesc->hyst_reset, &off, sizeof(off), hipMemcpyHostToDevice, s));
            HIPCHK(hipStreamSynchronize(s));
            if (rc != LBM_OK) return rc;
        }
        return LBM_OK;
    }
    if (init->kind != LBM_INIT_FIELDS || !init->phi) {
        set_error("FIELDS init needs phi"); return LBM_E_INVAL;
    }
    // phi: fluid nodes from the input, ghosts from their owners, solid 0
    std::vector<char> hphi((size_t)N * sphi, 0);
    const int nx = p->nx, ny = p->ny;
    for (int64_t n = 0; n < N; ++n) {
        const int kind = flag_kind(L.flag[n]);
        double v = 0.0;
        if (kind == KIND_FLUID) v = init->phi[n];
        else if (kind == KIND_GHOST) {
            const int face = flag_sub(L.flag[n]);
            const int ax = face / 2, sgn = (face & 1) ? -1 : 1;
            const int64_t stride = ax == 0 ? 1 : (ax == 1 ? nx : (int64_t)nx * ny);
            v = init->phi[n + sgn * stride];
        }
        if (sphi == 8) ((double*)hphi.data())[n] = v;
        else ((float*)hphi.data())[n] = (float)v;
    }
    HIPCHK(hipMemcpyAsync(base + L.off_phi, hphi.data(), hphi.size(), hipMemcpyHostToDevice, s));
    double *du = nullptr, *dP = nullptr;
    if (init->u) {
        HIPCHK(hipMalloc(&du, (size_t)3 * N * sizeof(double)));
        HIPCHK(hipMemcpyAsync(du, init->u, (size_t)3 * N * sizeof(double), hipMemcpyHostToDevice, s));
    }
    if (init->P) {
        HIPCHK(hipMalloc(&dP, (size_t)N * sizeof(double)));
        HIPCHK(hipMemcpyAsync(dP, init->P, (size_t)N * sizeof(double), hipMemcpyHostToDevice, s));
    }
    ReadOut ro = {nullptr, nullptr, nullptr, nullptr};
    InitIn in = {du, dP};
    hipError_t e = launch_wall(p->storage, MODE_INIT, ddesc, (const WallRef*)(base + L.off_wrefs),
                               (int)L.n_wall, s);
    if (e == hipSuccess) e = launch_sweep(p->storage, phase_q(p), MODE_INIT, L.tx, 0, ddesc, dtiles, nt, 0, ro, in, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (du) hipFree(du);
    if (dP) hipFree(dP);
    if (e != hipSuccess) { set_error("init kernel: %s", hipGetErrorString(e)); return LBM_E_DEVICE; }
    return LBM_OK;
}

// Doubles of device staging a read-back of this mask needs.
size_t read_staging_elems(const Desc& hdesc, uint32_t mask, const double* phi, const double* P,
                          const double* u, const double* pops) {
    const size_t N = (size_t)hdesc.N;
    const int qh = hdesc.q_phase == 19 ? 19 : 7;
    size_t nd = 0;
    if (phi && (mask & LBM_PHI)) nd += N;
    if (P && (mask & LBM_P)) nd += N;
    if (u && (mask & LBM_U)) nd += 3 * N;
    // the read kernel writes every population row: all of them are staged
    if (pops && (mask & (LBM_POP_H | LBM_POP_G))) nd += (size_t)(qh + QG) * N;
    return nd;
}

int read_lattice_staged(int storage, const Desc& hdesc, int parity, Desc* d_desc, const Tile* d_tiles,
                        int ntiles, const WallRef* d_walls, int nwalls, uint32_t mask, double* phi,
                        double* P, double* u, double* pops, double* buf, hipStream_t s) {
    const int64_t N = hdesc.N;
    const bool want_pop = (mask & (LBM_POP_H | LBM_POP_G)) && pops;
    const int qh = hdesc.q_phase == 19 ? 19 : 7;
    size_t nd = 0;
    const size_t o_phi = nd; if (phi && (mask & LBM_PHI)) nd += N;
    const size_t o_P = nd; if (P && (mask & LBM_P)) nd += N;
    const size_t o_u = nd; if (u && (mask & LBM_U)) nd += 3 * N;
    const size_t o_pop = nd; if (want_pop) nd += (size_t)(qh + QG) * N;
    ReadOut ro;
    ro.phi = (phi && (mask & LBM_PHI)) ? buf + o_phi : nullptr;
    ro.P = (P && (mask & LBM_P)) ? buf + o_P : nullptr;
    ro.u = (u && (mask & LBM_U)) ? buf + o_u : nullptr;
    ro.pops = want_pop ? buf + o_pop : nullptr;
    InitIn in = {nullptr, nullptr};
    // nodes of dropped (all-solid) tiles are written by no read kernel: they
    // read 0 from the cleared staging
    hipError_t e = launch_fill_zero(buf, (int64_t)nd, s);
    if (e == hipSuccess) e = launch_phi(storage, qh, parity, d_desc, d_tiles, ntiles, s, 1);
    if (e == hipSuccess) e = launch_wall(storage, MODE_READ, d_desc, d_walls, nwalls, s);
    if (e == hipSuccess) e = launch_sweep(storage, qh, MODE_READ, hdesc.tx, parity, d_desc, d_tiles, ntiles, 1, ro, in, s);
    if (e == hipSuccess && ro.phi) e = hipMemcpyAsync(phi, ro.phi, N * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && ro.P) e = hipMemcpyAsync(P, ro.P, N * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && ro.u) e = hipMemcpyAsync(u, ro.u, 3 * N * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && ro.pops) {
        double* dst = pops;
        if (mask & LBM_POP_H) {
            e = hipMemcpyAsync(dst, ro.pops, (size_t)qh * N * sizeof(double), hipMemcpyDeviceToHost, s);
            dst += (size_t)qh * N;
        }
        if (e == hipSuccess && (mask & LBM_POP_G))
            e = hipMemcpyAsync(dst, ro.pops + (size_t)qh * N, (size_t)QG * N * sizeof(double),
                               hipMemcpyDeviceToHost, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { set_error("read fields: %s", hipGetErrorString(e)); return LBM_E_DEVICE; }
    return LBM_OK;
}

int read_lattice(int storage, const Desc& hdesc, int parity, Desc* d_desc, const Tile* d_tiles,
                 int ntiles, const WallRef* d_walls, int nwalls, uint32_t mask, double* phi,
                 double* P, double* u, double* pops, hipStream_t s) {
    const size_t nd = read_staging_elems(hdesc, mask, phi, P, u, pops);
    double* buf = nullptr;
    if (nd) HIPCHK(hipMalloc(&buf, nd * sizeof(double)));
    const int rc = read_lattice_staged(storage, hdesc, parity, d_desc, d_tiles, ntiles, d_walls, nwalls,
                                       mask, phi, P, u, pops, buf, s);
    if (buf) hipFree(buf);
    return rc;
}

}  // namespace pflbm
