// Internal definitions of libsmcx shared by the host driver and the gfx950
// kernels: lattice geometry (compile-time shell tables), per-replica metadata
// and kernel argument blocks.
#pragma once

#include <stdint.h>

#include "smcx.h"

namespace smcx {

// Halo, in conventional cells, of the padded occupancy copy and of every tile
// window.  A pair-model trial reads within 1 + c_max <= 4 half-units of its
// site (c_max <= 3 for the first four BCC / FCC shells), which lies within
// two conventional cells on every axis.
constexpr int kHalo = 2;
constexpr int kMaxShells = 4;
constexpr int kMaxZ = 24;
constexpr int kMaxK = 8;
constexpr int kMaxZ1 = 12;
constexpr int kMaxSumZ = 54;
constexpr int kBlock = 256;
constexpr int kMaxRowBlock = 1024;  // row kernel: several x-rows of link cells per workgroup
// Static workspace of smcx_lattice_init_static (bytes, per device) and the
// device ordinals it serves.
constexpr size_t kStaticWorkspaceBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

// ---------------------------------------------------------------------------
// Geometry.  Positions are in half lattice constants.  Coordination shells are
// the lattice vectors of the s-th smallest non-zero length, in lexicographic
// (dx, dy, dz) order; the first shell lists the swap partners (Methods,
// "Search neighbors": neighbours are found from a list of relative
// positions).  Built at compile time by enumerating a small box.
// ---------------------------------------------------------------------------
struct Geometry {
    int m;
    int basis[4][3];
    int nshell;
    int r2[kMaxShells];
    int Z[kMaxShells];
    int v[kMaxShells][kMaxZ][3];
};

constexpr int parity(int a) { return a & 1; }  // two's complement: also right for a < 0

constexpr int basis_of_parity(const Geometry& g, int px, int py, int pz)
{
    for (int b = 0; b < g.m; ++b)
        if (g.basis[b][0] == px && g.basis[b][1] == py && g.basis[b][2] == pz) return b;
    return -1;
}

constexpr Geometry make_geometry(int lattice)
{
    Geometry g{};
    if (lattice == SMCX_BCC) {
        g.m = 2;
        g.basis[1][0] = g.basis[1][1] = g.basis[1][2] = 1;
    } else {
        g.m = 4;
        g.basis[1][0] = 1; g.basis[1][1] = 1;
        g.basis[2][0] = 1; g.basis[2][2] = 1;
        g.basis[3][1] = 1; g.basis[3][2] = 1;
    }
    g.nshell = 0;
    for (int r2 = 1; r2 < 32 && g.nshell < kMaxShells; ++r2) {
        int n = 0;
        for (int x = -3; x <= 3; ++x)
            for (int y = -3; y <= 3; ++y)
                for (int z = -3; z <= 3; ++z) {
                    if (x * x + y * y + z * z != r2) continue;
                    if (basis_of_parity(g, parity(x), parity(y), parity(z)) < 0) continue;
                    g.v[g.nshell][n][0] = x;
                    g.v[g.nshell][n][1] = y;
                    g.v[g.nshell][n][2] = z;
                    ++n;
                }
        if (n > 0) {
            g.r2[g.nshell] = r2;
            g.Z[g.nshell] = n;
            ++g.nshell;
        }
    }
    return g;
}

constexpr Geometry kGeom[2] = {make_geometry(SMCX_BCC), make_geometry(SMCX_FCC)};

// In lexicographic order the second half of a shell is the first half negated
// (in reverse), so the first half holds one vector of every +-d pair.
constexpr bool shells_pair_up(const Geometry& g)
{
    for (int s = 0; s < g.nshell; ++s)
        for (int n = 0; n < g.Z[s]; ++n)
            for (int a = 0; a < 3; ++a)
                if (g.v[s][g.Z[s] - 1 - n][a] != -g.v[s][n][a]) return false;
    return true;
}
static_assert(shells_pair_up(kGeom[0]) && shells_pair_up(kGeom[1]), "shells must be sorted lexicographically");

// Neighbour of a basis-b site by half-unit vector (vx, vy, vz): the target
// basis bt and the displacement (dx, dy, dz) of its conventional cell.
struct Nb {
    int dx, dy, dz, bt;
};

constexpr Nb nb_of(const Geometry& g, int b, int vx, int vy, int vz)
{
    const int hx = g.basis[b][0] + vx, hy = g.basis[b][1] + vy, hz = g.basis[b][2] + vz;
    const int bt = basis_of_parity(g, parity(hx), parity(hy), parity(hz));
    Nb n{};
    n.bt = bt;
    n.dx = (hx - g.basis[bt][0]) / 2;  // exact: the difference is even
    n.dy = (hy - g.basis[bt][1]) / 2;
    n.dz = (hz - g.basis[bt][2]) / 2;
    return n;
}

constexpr int max_component(const Geometry& g, int S)
{
    int c = 0;
    for (int s = 0; s < S; ++s)
        for (int n = 0; n < g.Z[s]; ++n)
            for (int a = 0; a < 3; ++a) {
                const int v = g.v[s][n][a] < 0 ? -g.v[s][n][a] : g.v[s][n][a];
                if (v > c) c = v;
            }
    return c;
}

constexpr int sum_Z(const Geometry& g, int S)
{
    int t = 0;
    for (int s = 0; s < S; ++s) t += g.Z[s];
    return t;
}

static_assert(kGeom[0].Z[0] == 8 && kGeom[0].Z[1] == 6 && kGeom[0].Z[2] == 12 && kGeom[0].Z[3] == 24,
              "BCC coordination numbers");
static_assert(kGeom[1].Z[0] == 12 && kGeom[1].Z[1] == 6 && kGeom[1].Z[2] == 24 && kGeom[1].Z[3] == 12,
              "FCC coordination numbers");
static_assert(max_component(kGeom[0], 4) == 3 && max_component(kGeom[1], 4) == 2, "shell reach");

// ---------------------------------------------------------------------------
// Per-replica metadata, stored in the workspace.
// Padded copy: conventional cell x in [-kHalo, L + kHalo) on every axis; byte
// of site (x, y, z, b) = pad_off + ((z + H) * prows + (y + H)) * prow
//                        + m * (x + H) + b.
// ---------------------------------------------------------------------------
struct RepDev {
    int32_t L[3];        // conventional cells per axis
    int32_t nc[3];       // link cells per axis
    int32_t M[3];        // largest link-cell edge per axis
    int32_t emin[3];     // smallest link-cell edge per axis
    int32_t nA;          // mini-steps per sweep
    int32_t ntile[3];    // tiles per axis
    int32_t cs_off;      // cell-origin table offset (x: nc0+1 entries, then y, then z)
    int32_t prow;        // padded row pitch (bytes, multiple of 16)
    int32_t prows;       // rows per padded plane (L1 + 2H)
    int32_t alias;       // some partner has images in another shell (an edge of 2)
    int32_t rg[2];       // row kernel: groups of rows along y and z
    int32_t cp;          // basis-planar padded copy (row kernel): column pitch, bytes per basis site
    int32_t prowp;       // basis-planar padded copy: row pitch (m * cp)
    int64_t pad_off;     // byte offset of the padded copy in the workspace
    int64_t occ_off;     // first site of this replica in the occupancy array
    int64_t N;           // sites
    int64_t ntiles;      // tiles per mini-step
    uint8_t mult[kMaxShells][kMaxZ1];  // images of the partner inside each shell
};

// ---------------------------------------------------------------------------
// Compile-time window presets for uniform partitions (every link cell of edge
// ELL).  A tile of TX x TY x TZ cells starting at cell c0 and mini-step
// offsets o stages conventional cells c0*ELL + o - H .. + ELL*(T-1) + 2H on
// each axis; along x the staged bytes are 16-byte aligned, which for
// TX*ELL*m divisible by 16 starts at floor16(m*o) past the tile origin.
// ---------------------------------------------------------------------------
struct Preset {
    int lattice, tx, ty, tz, ell, K, S;
};

constexpr Preset kPresets[] = {
    {SMCX_BCC, 16, 4, 4, 4, 4, 4},  // 4-component BCC alloy, 4 shells
    {SMCX_BCC, 16, 4, 2, 4, 4, 4},
    {SMCX_FCC, 16, 4, 2, 4, 5, 4},  // 5-component FCC alloy, 4 shells
    {SMCX_FCC, 8, 4, 4, 4, 5, 4},
};
constexpr int kNumPresets = sizeof(kPresets) / sizeof(kPresets[0]);

// Compile-time row windows (row kernel): column pitch, window row pitch and
// depths, lanes (cells along x, rows along y and z) and species / shells.
// With them every neighbour offset in the window is a constant.
struct RowPreset {
    int lattice, K, S, cp, LP, WY, WZ, rt0, rt1, rt2;
};
constexpr RowPreset kRowPresets[] = {
    {SMCX_BCC, 4, 4, 816, 1664, 5, 9, 200, 1, 2},  // 800-cell rows, link cells of 4, 1 x 2 rows per workgroup
    // the paper's large lattice, 795-cell rows (Tab. 4): 4 shells with link
    // cells of 4 and 5, and 2 shells with link cells of 3; one row per workgroup
    {SMCX_BCC, 4, 4, 800, 1792, 5, 5, 198, 1, 1},
    {SMCX_BCC, 4, 2, 800, 1792, 5, 5, 265, 1, 1},
};
constexpr int kNumRowPresets = sizeof(kRowPresets) / sizeof(kRowPresets[0]);

constexpr int preset_m(const Preset& p) { return p.lattice == SMCX_BCC ? 2 : 4; }
constexpr int preset_w(int t, int ell) { return ell * (t - 1) + 1 + 2 * kHalo; }
constexpr int preset_LP(const Preset& p)
{
    const int m = preset_m(p);
    int best = 0;
    for (int o = 0; o < p.ell; ++o) {
        const int lo = (m * o) & ~15;
        const int hi = (m * (o + preset_w(p.tx, p.ell)) + 15) & ~15;
        if (hi - lo > best) best = hi - lo;
    }
    return best;
}
constexpr int preset_WY(const Preset& p) { return preset_w(p.ty, p.ell); }
constexpr int preset_WZ(const Preset& p) { return preset_w(p.tz, p.ell); }
constexpr bool preset_ok(const Preset& p) { return (p.tx * p.ell * preset_m(p)) % 16 == 0; }

// Arguments of the sweep kernels (passed by value).
struct SweepArgs {
    const RepDev* reps;
    const int32_t* origins;
    const int64_t* tile_off;   // [R + 1] prefix sums of tiles per replica
    const int16_t* offP;       // [m][Z1][sumZ] partner-neighbour offsets relative to the active site
    const int32_t* offB;       // [m][Z1] partner offset relative to the active site
    const int8_t* pdisp;       // [m][Z1][4] partner cell displacement and basis
    const double* Dtab;        // [S][K][K][K]: D[s][t][p][q] = V_s[q][t] - V_s[p][t]
    const int32_t* Qtab;       // [S][K][K][K] D in integer units, [K][K] bias sums, then the unit and
                               // the error bound as float bits (qtab_entries + 2 words)
    uint8_t* ws;               // workspace base (padded copies)
    const double* beta;        // beta[js * beta_stride + r]
    int64_t* stats;            // [R][3]
    smcx_tie* ties;
    int32_t* tie_count;
    const uint32_t* sweep_counter;  // when set, first sweep index is read here
    uint64_t seed;
    uint32_t first_sweep;
    int32_t n_sweeps;
    int32_t beta_stride;
    int32_t tie_cap;
    int32_t R, K, S, Z1, sumZ;
    int32_t T[3];              // tile shape (link cells)
    int32_t LP, WY, WZ;        // LDS window: row pitch, rows per plane, planes
    int32_t lds_d, lds_q, lds_offp, lds_offb, lds_pd, lds_win;  // dynamic-LDS byte offsets
    int32_t win_bytes;         // one window buffer
    int32_t nbuf;              // window buffers: 2 = next tile streams in during the trials, 1 = staged in turn
    int32_t g;                 // mini-step (stream / plain launches)
    int32_t gq;                // row launches over replicas of different decompositions: group index q
                               // (every replica runs its q-th (o_y, o_z) group, all offsets), else -1
    int32_t nb;                // stream / plain: mini-steps g .. g + nb - 1 (one offset o, consecutive basis
                               // sites) share one staged window; persistent: the group size (1 or m)
    int32_t tau_begin, tau_end; // persistent launches: mini-step range of every sweep
    int32_t only_rep;          // plain launches: the replica, else -1
};

// Dynamic LDS layout helpers (byte offsets, 16-aligned).
struct LdsLayout {
    int d_off, q_off, offp_off, offb_off, pd_off, win_off, win_bytes, total;
};

// Entries of the integer dE table: [S][K][K][K] terms, then [K][K] bias sums
// (two float words follow them in memory: the unit and the error bound).
inline int qtab_entries(int K, int S) { return S * K * K * K + K * K; }

inline LdsLayout lds_layout(int lattice, int K, int S, int Z1, int sumZ, int win_bytes, int nbuf)
{
    auto al = [](int v) { return (v + 15) & ~15; };
    const int m = lattice == SMCX_BCC ? 2 : 4;
    LdsLayout L{};
    int o = 0;
    L.d_off = o;    o = al(o + 8 * K * K * S * K);
    L.q_off = o;    o = al(o + 4 * qtab_entries(K, S));
    // the partner-neighbour offset table serves FCC windows only
    L.offp_off = o; o = al(o + (lattice == SMCX_FCC ? 2 * m * Z1 * sumZ : 0));
    L.offb_off = o; o = al(o + 4 * m * Z1);
    L.pd_off = o;   o = al(o + 4 * m * Z1);
    L.win_off = o;
    L.win_bytes = al(win_bytes);
    o = al(o + nbuf * L.win_bytes);
    L.total = o;
    return L;
}

}  // namespace smcx
