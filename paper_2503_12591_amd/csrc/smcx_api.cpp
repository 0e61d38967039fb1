// C ABI of libsmcx (declared in include/smcx.h): argument checking, the
// partition and launch plan, workspace layout, table upload and the sweep
// drivers.  Everything that touches lattice sites runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "smcx.h"
#include "smcx_internal.h"
#include "smcx_launch.h"

using namespace smcx;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

#define SMCX_HIP(call)                                                                              \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess) return fail(SMCX_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int lattice_m(int lattice) { return lattice == SMCX_BCC ? 2 : 4; }

// Minimum link-cell edge: trials read within 1 + c_max half-units of their
// site and write within 1; active sites of one mini-step are >= 2*ell apart
// on some axis.  (Link cells larger than the interaction range, Methods,
// link-cell bullet; LIZ / LIZ+ regions, Results and Fig. 1c.)
int min_edge(int lattice, int S)
{
    const int c = max_component(kGeom[lattice], S);
    int ell = 1;
    while (!(2 * ell > 2 + c)) ++ell;
    return ell;
}

// Smallest cell edge for which the trials of consecutive basis sites at one
// offset may share a staged window: a lane's next site moves by up to one
// half-lattice unit per axis, so other cells' written sites (within one unit
// of their active sites) must stay beyond the read reach 1 + c_max of it:
// 2 * ell - 1 > 2 + c_max.  The same bound keeps periodic images of a
// written site out of that reach.
int group_edge(int lattice, int S)
{
    const int c = max_component(kGeom[lattice], S);
    int ell = 1;
    while (!(2 * ell > 3 + c)) ++ell;
    return ell;
}

struct Replica {
    int L[3];
    std::vector<int> edges[3];
    std::vector<int> origin[3];  // nc + 1 entries
    int M[3];
    int nA;
    int64_t N;
    int64_t occ_off;
    int ntile[3];
    int64_t ntiles;
    int prow, prows;
    int cp, prowp;  // basis-planar rows: column pitch and row pitch
    int64_t pad_off, pad_bytes;
    int mult[kMaxShells][kMaxZ1];
    int rg[2];  // row kernel: row groups along y and z
};

struct Plan {
    int lattice, K, S, R, m, Z1, sumZ;
    int T[3];
    int block;  // threads per workgroup: the tile's link cells rounded up to whole waves
    int nbuf;   // window buffers per workgroup
    int group;  // mini-steps of consecutive basis sites sharing one staged window (m, or 1 if an edge < 4)
    // row kernel (stream mode): lanes = RT[0] cells along x times RT[1] x RT[2] rows
    bool rows;
    bool rows_mixed;  // replicas differ in mini-step decomposition: row launches only for whole sweeps
    int RT[3], rblock, rLP, rWY, rWZ;
    int row_preset;  // compile-time row window matching the plan, or -1
    LdsLayout rlds;
    size_t off_rowoff, off_offP_r, off_offB_r;
    int64_t total_rowgroups;
    int preset; // compile-time window preset of the stream kernel, or -1
    std::vector<Replica> reps;
    int LP, WY, WZ;
    LdsLayout lds;
    size_t off_reps, off_origins, off_tileoff, off_offP, off_offB, off_pd, off_D, off_Q, off_V, off_misc, off_pad, total;
    // qSRO model: affected-set and neighbour tables, V, W, Z
    size_t off_qaff, off_qnbr, off_qV, off_qW, off_qZ, off_qslots;
    int qnaff;   // largest affected set
    int qreach;  // cells per axis from the active site's cell to the farthest site a qSRO trial reads
    int n_origins;
    int64_t total_sites, total_tiles;
    int max_nA;
};

// Worst LDS bank sharing of a row window's lanes: lanes walk x fastest, then
// the ry rows of cells, then the rz planes of cells; a lane's site byte is
// ell (x) + ell * prow (y) + ell * prow * wy (z) from its neighbour's, and a
// wave's 64 lanes read 64 banks of 4 bytes.  Returns the largest number of
// lanes of one wave in one bank (1: conflict-free).
static int row_bank_ways(int ncx, int ry, int rz, int prow, int wy, int ell)
{
    const int lanes = ncx * ry * rz;
    int worst = 1;
    for (int w0 = 0; w0 < lanes; w0 += 64) {
        int count[64] = {0};
        for (int g = w0; g < std::min(lanes, w0 + 64); ++g) {
            const int lx = g % ncx, ly = (g / ncx) % ry, lz = g / (ncx * ry);
            const int64_t byte = (int64_t)ell * lx + (int64_t)ell * prow * (ly + (int64_t)wy * lz);
            worst = std::max(worst, ++count[(byte >> 2) & 63]);
        }
    }
    return worst;
}

int make_plan(const smcx_desc* d, Plan& P)
{
    if (!d) return fail(SMCX_E_INVALID_ARG, "desc is NULL");
    if (d->lattice != SMCX_BCC && d->lattice != SMCX_FCC) return fail(SMCX_E_INVALID_ARG, "lattice must be SMCX_BCC or SMCX_FCC");
    if (d->n_species < 2 || d->n_species > kMaxK) return fail(SMCX_E_INVALID_ARG, "n_species must be in 2..8");
    if (d->n_shells < 1 || d->n_shells > kMaxShells) return fail(SMCX_E_INVALID_ARG, "n_shells must be in 1..4");
    if (d->n_replicas < 1) return fail(SMCX_E_INVALID_ARG, "n_replicas must be >= 1");
    if (!d->dims) return fail(SMCX_E_INVALID_ARG, "dims is NULL");
    if ((d->ncell == nullptr) != (d->cells == nullptr)) return fail(SMCX_E_INVALID_ARG, "ncell and cells must both be set or both NULL");
    if (d->flags & ~(uint32_t)(SMCX_FLAG_DOUBLE_BUFFER | SMCX_FLAG_TILES)) return fail(SMCX_E_INVALID_ARG, "unknown flags");
    P.nbuf = (d->flags & SMCX_FLAG_DOUBLE_BUFFER) ? 2 : 1;
    P.lattice = d->lattice;
    P.K = d->n_species;
    P.S = d->n_shells;
    P.R = d->n_replicas;
    P.m = lattice_m(P.lattice);
    P.group = P.m;
    const int gedge = group_edge(P.lattice, d->n_shells);
    const Geometry& G = kGeom[P.lattice];
    P.Z1 = G.Z[0];
    P.sumZ = sum_Z(G, P.S);
    const int emin = min_edge(P.lattice, P.S);
    if (d->tile[0] == 0 && d->tile[1] == 0 && d->tile[2] == 0) {
        P.T[0] = 16; P.T[1] = 4; P.T[2] = 2;
    } else {
        for (int a = 0; a < 3; ++a) {
            if (d->tile[a] < 1) return fail(SMCX_E_INVALID_ARG, "tile edges must be >= 1");
            P.T[a] = d->tile[a];
        }
        if ((int64_t)P.T[0] * P.T[1] * P.T[2] > kBlock) return fail(SMCX_E_INVALID_ARG, "tile holds more than 256 link cells");
    }
    P.block = (P.T[0] * P.T[1] * P.T[2] + 63) / 64 * 64;
    P.reps.resize(P.R);
    int64_t occ_off = 0;
    size_t cells_pos = 0;
    P.max_nA = 0;
    for (int r = 0; r < P.R; ++r) {
        Replica& R = P.reps[r];
        for (int a = 0; a < 3; ++a) {
            R.L[a] = d->dims[3 * r + a];
            if (R.L[a] < 2) return fail(SMCX_E_INVALID_ARG, "every dimension must be >= 2 (replica " + std::to_string(r) + ")");
            if (R.L[a] > (1 << 20)) return fail(SMCX_E_UNSUPPORTED, "dimension too large");
        }
        // no neighbour vector may map a site onto itself
        for (int s = 0; s < P.S; ++s)
            for (int n = 0; n < G.Z[s]; ++n) {
                bool self = true;
                for (int a = 0; a < 3; ++a) self &= (G.v[s][n][a] % (2 * R.L[a])) == 0;
                if (self) return fail(SMCX_E_INVALID_ARG, "lattice too small: a site would be its own neighbour");
            }
        const int64_t ncell = (int64_t)R.L[0] * R.L[1] * R.L[2];
        if (ncell > 0x7fffffffLL) return fail(SMCX_E_UNSUPPORTED, "more than 2^31 conventional cells in one replica");
        R.N = ncell * P.m;
        R.occ_off = occ_off;
        occ_off += R.N;
        for (int a = 0; a < 3; ++a) {
            R.edges[a].clear();
            if (d->cells) {
                const int nc = d->ncell[3 * r + a];
                if (nc < 1 || nc > R.L[a]) return fail(SMCX_E_INVALID_ARG, "bad ncell");
                int sum = 0;
                for (int j = 0; j < nc; ++j) {
                    const int e = d->cells[cells_pos++];
                    if (e < 1) return fail(SMCX_E_INVALID_ARG, "cell edges must be >= 1");
                    R.edges[a].push_back(e);
                    sum += e;
                }
                if (sum != R.L[a]) return fail(SMCX_E_INVALID_ARG, "cell edges do not sum to the dimension");
            } else {
                int ell = d->ell ? d->ell[r] : 4;
                if (ell < 1) return fail(SMCX_E_INVALID_ARG, "ell must be >= 1");
                ell = std::max(ell, emin);
                const int n = std::max(1, R.L[a] / ell);
                for (int j = 0; j < n; ++j) R.edges[a].push_back(R.L[a] / n + (j < R.L[a] % n ? 1 : 0));
            }
            if (R.edges[a].size() > 1)
                for (int e : R.edges[a])
                    if (e < emin)
                        return fail(SMCX_E_INVALID_ARG, "link-cell edge " + std::to_string(e) + " below the minimum " +
                                                            std::to_string(emin) + " for independent trials");
            R.origin[a].assign(1, 0);
            R.M[a] = 0;
            for (int e : R.edges[a]) {
                R.origin[a].push_back(R.origin[a].back() + e);
                R.M[a] = std::max(R.M[a], e);
                if (e < gedge) P.group = 1;
            }
            R.ntile[a] = ((int)R.edges[a].size() + P.T[a] - 1) / P.T[a];
        }
        R.nA = R.M[0] * R.M[1] * R.M[2] * P.m;
        P.max_nA = std::max(P.max_nA, R.nA);
        R.ntiles = (int64_t)R.ntile[0] * R.ntile[1] * R.ntile[2];
        R.prow = (P.m * (R.L[0] + 2 * kHalo) + 15) & ~15;
        R.cp = (R.L[0] + 2 * kHalo + 15) & ~15;
        R.prowp = P.m * R.cp;
        R.prows = R.L[1] + 2 * kHalo;
        // one region serves both layouts (a sweep call packs the one its kernels read)
        R.pad_bytes = (int64_t)std::max(R.prow, R.prowp) * R.prows * (R.L[2] + 2 * kHalo);
        // partner images inside each shell: #{d in D_s : d == D_1[k] mod 2L}
        for (int s = 0; s < kMaxShells; ++s)
            for (int k = 0; k < kMaxZ1; ++k) R.mult[s][k] = 0;
        for (int k = 0; k < P.Z1; ++k)
            for (int s = 0; s < P.S; ++s)
                for (int n = 0; n < G.Z[s]; ++n) {
                    bool same = true;
                    for (int a = 0; a < 3; ++a) same &= ((G.v[s][n][a] - G.v[0][k][a]) % (2 * R.L[a])) == 0;
                    R.mult[s][k] += same ? 1 : 0;
                }
    }
    if (d->cells) {
        // nothing else to check: positions were consumed replica by replica
    }
    P.total_sites = occ_off;

    // LDS window extents over every tile and offset (per axis independently)
    int maxn[3] = {0, 0, 0};
    int maxbytes = 0;
    for (const Replica& R : P.reps)
        for (int a = 0; a < 3; ++a) {
            const int nc = (int)R.edges[a].size();
            for (int ti = 0; ti < R.ntile[a]; ++ti) {
                const int c0 = ti * P.T[a];
                const int c1 = std::min(c0 + P.T[a], nc);
                for (int o = 0; o < R.M[a]; ++o) {
                    const int w0 = R.origin[a][c0] + o - kHalo;
                    const int w1 = std::min(R.origin[a][c1 - 1] + o + kHalo + 1, R.L[a] + kHalo);
                    if (w1 <= w0) continue;
                    maxn[a] = std::max(maxn[a], w1 - w0);
                    if (a == 0) {
                        const int gx0 = (P.m * (w0 + kHalo)) & ~15;
                        const int gx1 = (P.m * (w1 + kHalo) + 15) & ~15;
                        maxbytes = std::max(maxbytes, gx1 - gx0);
                    }
                }
            }
        }
    P.LP = maxbytes;
    P.WY = maxn[1];
    P.WZ = maxn[2];
    // a compile-time window applies when every replica is cut into uniform
    // cells of the preset's edge and the tile matches; its (larger or equal)
    // window dimensions then define the LDS layout and the offset tables
    P.preset = -1;
    for (int pi = 0; pi < kNumPresets && P.preset < 0; ++pi) {
        const Preset& q = kPresets[pi];
        if (q.lattice != P.lattice || q.tx != P.T[0] || q.ty != P.T[1] || q.tz != P.T[2]) continue;
        if (P.LP > preset_LP(q) || P.WY > preset_WY(q) || P.WZ > preset_WZ(q)) continue;
        bool uniform = true;
        for (const Replica& R : P.reps)
            for (int a = 0; a < 3; ++a)
                for (int e : R.edges[a]) uniform &= e == q.ell;
        if (!uniform || P.K != q.K || P.S != q.S || P.nbuf != 1) continue;
        P.preset = pi;
        P.LP = preset_LP(q);
        P.WY = preset_WY(q);
        P.WZ = preset_WZ(q);
    }
    if (P.LP > 4096) return fail(SMCX_E_UNSUPPORTED, "tile window rows longer than 4096 bytes; use a smaller tile");
    const int64_t win = (int64_t)P.LP * P.WY * P.WZ;
    if (win > 160 * 1024) return fail(SMCX_E_UNSUPPORTED, "tile window does not fit in LDS; use a smaller tile");
    P.lds = lds_layout(P.lattice, P.K, P.S, P.Z1, P.sumZ, (int)win, P.nbuf);
    if (P.lds.total > 160 * 1024) return fail(SMCX_E_UNSUPPORTED, "tile window and tables exceed 160 KiB of LDS");
    const int64_t max_off = 2LL * P.LP * P.WY + 2LL * P.LP + 2 * P.m + 4;
    if (max_off > 32767) return fail(SMCX_E_UNSUPPORTED, "LDS offsets exceed 16 bits; use a smaller tile");

    // row kernel: whole x-rows per workgroup, every o_x of a (o_y, o_z) group
    // in one launch.  Needs shared windows for all basis sites (P.group), the
    // same mini-step decomposition in every replica, a row within one block,
    // and windows no taller than the lattice on y and z (so no site appears
    // twice in a window except through the x halo).
    P.rows = false;
    P.rows_mixed = false;
    P.row_preset = -1;
    if (P.group == P.m && P.nbuf == 1 && !(d->flags & SMCX_FLAG_TILES)) {
        bool same_m = true, same_cp = true;
        // basis-planar rows in the window; a pitch that is a multiple of 256
        // bytes keeps lanes' partner reads in the banks of their own sites, a
        // multiple of 128 costs a few two-way conflicts but may let one more
        // workgroup fit per CU
        int ncx = 0, prowp = 0;
        for (const Replica& R : P.reps) {
            for (int a = 0; a < 3; ++a) same_m &= R.M[a] == P.reps[0].M[a];
            ncx = std::max(ncx, (int)R.edges[0].size());
            prowp = std::max(prowp, R.prowp);
            same_cp &= R.cp == P.reps[0].cp;
        }
        // score: busy lanes per block x waves per CU (12 make up for latency)
        // x a penalty when a single workgroup per CU leaves its staging
        // exposed x a small one for the 128-byte pitch
        const int tables = lds_layout(P.lattice, P.K, P.S, P.Z1, P.sumZ, 0, 1).total;
        double best_score = 0.0;
        int best_lanes = 0, best_win = 0, best_prow = 0, best[4] = {0, 0, 0, 0};
        // FCC partners count through a table of window offsets, which holds one
        // column pitch; BCC partners derive theirs per replica
        P.rows_mixed = !same_m;
        // Short rows (fewer cells than a wave has lanes) put several cell
        // rows in one wave; their sites sit ell pitches apart in y and ell
        // plane strides apart in z, so a pitch that is a multiple of 256
        // bytes maps them all to the same LDS banks.  For BCC replicas of one
        // decomposition, pitches in 16-byte steps are tried too, scored by
        // the worst bank sharing (measured: 256 BCC 32^3 replicas 1.57e10 ->
        // 1.74e10 swaps/s; a ladder of mixed sizes and FCC 128^3 ran slower
        // with it, so they keep the aligned pitches).
        std::vector<int> pitches = {(prowp + 255) & ~255, (prowp + 127) & ~127};
        const bool short_rows = ncx < 64 && P.lattice == SMCX_BCC && same_m;
        if (short_rows)
            for (int t = 0; t < 8; ++t) pitches.push_back(((prowp + 15) & ~15) + 16 * t);
        std::sort(pitches.begin(), pitches.end());
        pitches.erase(std::unique(pitches.begin(), pitches.end()), pitches.end());
        // x strides of the cells the replicas have (edges differ by at most one)
        int ell_lo = 1 << 30, ell_hi = 0;
        for (const Replica& R : P.reps)
            for (int e : R.edges[0]) {
                ell_lo = std::min(ell_lo, e);
                ell_hi = std::max(ell_hi, e);
            }
        if ((same_cp || P.lattice == SMCX_BCC) && ncx <= kMaxRowBlock)
          for (int prow : pitches)
            for (int ry : {1, 2, 4, 8, 16})
                for (int rz : {1, 2, 4, 8, 16}) {
                    const int lanes = ncx * ry * rz;
                    if (lanes > kMaxRowBlock) continue;
                    int wy = 0, wz = 0;
                    bool fits = true;
                    for (const Replica& R : P.reps) {
                        int wyr = 0, wzr = 0;
                        const int ncy = (int)R.edges[1].size(), ncz = (int)R.edges[2].size();
                        for (int c0 = 0; c0 < ncy; c0 += ry)
                            wyr = std::max(wyr, R.origin[1][std::min(c0 + ry, ncy) - 1] - R.origin[1][c0] + 1 + 2 * kHalo);
                        for (int c0 = 0; c0 < ncz; c0 += rz)
                            wzr = std::max(wzr, R.origin[2][std::min(c0 + rz, ncz) - 1] - R.origin[2][c0] + 1 + 2 * kHalo);
                        fits &= wyr <= R.L[1] && wzr <= R.L[2];
                        wy = std::max(wy, wyr);
                        wz = std::max(wz, wzr);
                    }
                    const int winb = prow * wy * wz;
                    // FCC partners count through a table of 16-bit window offsets
                    if (!fits || (P.lattice == SMCX_FCC &&
                                  2LL * prow * wy + 2LL * prow + (P.m + 1) * (int64_t)P.reps[0].cp > 32767))
                        continue;
                    const int lds = tables + ((winb + 15) & ~15);
                    if (lds > 160 * 1024) continue;
                    const int block = (lanes + 63) / 64 * 64;
                    const int waves = block / 64;
                    const int wave_cap = block <= kBlock ? 12 : 16;  // register budget of the instantiation
                    const int wgs = std::min(160 * 1024 / lds, wave_cap / waves);
                    if (wgs < 1) continue;
                    const int ways = short_rows ? std::max(row_bank_ways(ncx, ry, rz, prow, wy, ell_lo),
                                                           row_bank_ways(ncx, ry, rz, prow, wy, ell_hi))
                                                : 1;
                    const double banks = short_rows ? 1.0 / (0.75 + 0.25 * ways) : (prow % 256 ? 0.98 : 1.0);
                    const double score = (double)lanes / block * std::min(1.0, wgs * waves / 12.0) *
                                         (wgs == 1 ? 0.88 : 1.0) * banks;
                    if (score > best_score + 1e-12 || (std::fabs(score - best_score) <= 1e-12 && winb < best_win)) {
                        best_score = score;
                        best_lanes = lanes;
                        best_win = winb;
                        best_prow = prow;
                        best[0] = ry; best[1] = rz; best[2] = wy; best[3] = wz;
                    }
                }
        if (best_lanes > 0) {
            P.rows = true;
            P.RT[0] = ncx;
            P.RT[1] = best[0];
            P.RT[2] = best[1];
            P.rblock = (best_lanes + 63) / 64 * 64;
            P.rLP = best_prow;
            P.rWY = best[2];
            P.rWZ = best[3];
            P.rlds = lds_layout(P.lattice, P.K, P.S, P.Z1, P.sumZ, best_win, 1);
            P.row_preset = -1;
            // presets assume no partner has images in other shells
            bool images = false;
            for (const Replica& R : P.reps)
                for (int s = 0; s < kMaxShells; ++s)
                    for (int k = 0; k < P.Z1; ++k) images |= R.mult[s][k] != (s == 0 ? 1 : 0);
            for (int pi = 0; pi < kNumRowPresets; ++pi) {
                const RowPreset& q = kRowPresets[pi];
                if (same_cp && !images && q.lattice == P.lattice && q.K == P.K && q.S == P.S && q.cp == P.reps[0].cp && q.LP == P.rLP &&
                    q.WY == P.rWY && q.WZ == P.rWZ && q.rt0 == P.RT[0] && q.rt1 == P.RT[1] && q.rt2 == P.RT[2])
                    P.row_preset = pi;
            }
            P.total_rowgroups = 0;
            for (Replica& R : P.reps) {
                R.rg[0] = ((int)R.edges[1].size() + P.RT[1] - 1) / P.RT[1];
                R.rg[1] = ((int)R.edges[2].size() + P.RT[2] - 1) / P.RT[2];
                P.total_rowgroups += (int64_t)R.rg[0] * R.rg[1];
            }
        }
    }

    // workspace layout
    size_t o = 0;
    P.off_reps = o; o = align256(o + sizeof(RepDev) * P.R);
    P.n_origins = 0;
    for (const Replica& R : P.reps)
        for (int a = 0; a < 3; ++a) P.n_origins += (int)R.origin[a].size();
    P.off_origins = o; o = align256(o + sizeof(int32_t) * P.n_origins);
    P.off_tileoff = o; o = align256(o + sizeof(int64_t) * (P.R + 1));
    P.off_offP = o; o = align256(o + sizeof(int16_t) * P.m * P.Z1 * P.sumZ);
    P.off_offB = o; o = align256(o + sizeof(int32_t) * P.m * P.Z1);
    P.off_pd = o; o = align256(o + 4 * P.m * P.Z1);
    P.off_D = o; o = align256(o + sizeof(double) * P.K * P.K * P.S * P.K);
    P.off_Q = o; o = align256(o + sizeof(int32_t) * (qtab_entries(P.K, P.S) + 2));
    P.off_V = o; o = align256(o + sizeof(double) * P.S * P.K * P.K);
    P.off_misc = o; o = align256(o + 256);
    P.off_qaff = o; o = align256(o + sizeof(int32_t) * P.m * P.Z1 * (1 + kQsroMaxAff));
    P.off_qnbr = o; o = align256(o + sizeof(int32_t) * P.m * P.sumZ);
    P.off_qV = o; o = align256(o + sizeof(double) * P.S * P.K * P.K);
    P.off_qW = o; o = align256(o + sizeof(double) * P.S * P.K);
    P.off_qZ = o; o = align256(o + sizeof(int32_t) * kMaxShells);
    P.off_qslots = o; o = align256(o + sizeof(int64_t) * 3 * kQsroGrid);
    P.off_rowoff = o; o = align256(o + sizeof(int64_t) * (P.R + 1));
    P.off_offP_r = o; o = align256(o + sizeof(int16_t) * P.m * P.Z1 * P.sumZ);
    P.off_offB_r = o; o = align256(o + sizeof(int32_t) * P.m * P.Z1);
    P.off_pad = o;
    P.total_tiles = 0;
    for (Replica& R : P.reps) {
        R.pad_off = (int64_t)o;
        o = align256(o + (size_t)R.pad_bytes);
        P.total_tiles += R.ntiles;
    }
    P.total = o;
    return SMCX_OK;
}

// LDS offset of the site at half-unit vector v from a basis-b site in a
// window of row pitch LP and WY rows per plane.
int lds_offset(const Plan& P, int LP, int WY, int b, int vx, int vy, int vz)
{
    const Nb nb = nb_of(kGeom[P.lattice], b, vx, vy, vz);
    return nb.dz * LP * WY + nb.dy * LP + P.m * nb.dx + (nb.bt - b);
}

// Same in a window of basis-planar rows with column pitch cp.
int lds_offset_planar(const Plan& P, int LP, int WY, int cp, int b, int vx, int vy, int vz)
{
    const Nb nb = nb_of(kGeom[P.lattice], b, vx, vy, vz);
    return nb.dz * LP * WY + nb.dy * LP + nb.dx + (nb.bt - b) * cp;
}

}  // namespace

struct smcx_lattice {
    Plan P;
    uint8_t* occ;
    uint8_t* ws;
    size_t ws_bytes;
    bool epi_set = false;
    bool qsro_set = false;
    std::vector<double> V;       // [S][K][K]
    std::vector<double> Dhost;   // [S][K][K][K]: D[s][t][p][q]
    std::vector<int32_t> Qhost;  // D in integer units, the bias sums, the unit and the error bound (float bits)
    std::vector<int64_t> counts_host;
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    std::vector<hipEvent_t> pool;
    int64_t timed_launches = 0;
    int stream_wgs = 8;  // stream-mode grid: 8 XCD chunks x workgroups per XCD
    const void* k_stream = nullptr;
    const void* k_persistent = nullptr;
    const void* k_rows = nullptr;
    int rows_wgs = 8;
    int static_dev = -1;  // device whose static workspace this handle uses, else -1
};

namespace {

SweepArgs base_args(smcx_lattice* h)
{
    const Plan& P = h->P;
    SweepArgs a{};
    a.reps = (const RepDev*)(h->ws + P.off_reps);
    a.origins = (const int32_t*)(h->ws + P.off_origins);
    a.tile_off = (const int64_t*)(h->ws + P.off_tileoff);
    a.offP = (const int16_t*)(h->ws + P.off_offP);
    a.offB = (const int32_t*)(h->ws + P.off_offB);
    a.pdisp = (const int8_t*)(h->ws + P.off_pd);
    a.Dtab = (const double*)(h->ws + P.off_D);
    a.Qtab = (const int32_t*)(h->ws + P.off_Q);
    a.ws = h->ws;
    a.R = P.R;
    a.K = P.K;
    a.S = P.S;
    a.Z1 = P.Z1;
    a.sumZ = P.sumZ;
    for (int i = 0; i < 3; ++i) a.T[i] = P.T[i];
    a.LP = P.LP;
    a.WY = P.WY;
    a.WZ = P.WZ;
    a.lds_d = P.lds.d_off;
    a.lds_q = P.lds.q_off;
    a.lds_offp = P.lds.offp_off;
    a.lds_offb = P.lds.offb_off;
    a.lds_pd = P.lds.pd_off;
    a.lds_win = P.lds.win_off;
    a.win_bytes = P.lds.win_bytes;
    a.nbuf = P.nbuf;
    a.only_rep = -1;
    a.nb = 1;
    a.gq = -1;
    a.sweep_counter = nullptr;
    return a;
}

// Launch arguments of the row kernel: row windows, their offset tables and
// the prefix sums of row groups per replica.
SweepArgs row_args(smcx_lattice* h)
{
    const Plan& P = h->P;
    SweepArgs a = base_args(h);
    a.tile_off = (const int64_t*)(h->ws + P.off_rowoff);
    a.offP = (const int16_t*)(h->ws + P.off_offP_r);
    a.offB = (const int32_t*)(h->ws + P.off_offB_r);
    for (int i = 0; i < 3; ++i) a.T[i] = P.RT[i];
    a.LP = P.rLP;
    a.WY = P.rWY;
    a.WZ = P.rWZ;
    a.lds_d = P.rlds.d_off;
    a.lds_q = P.rlds.q_off;
    a.lds_offp = P.rlds.offp_off;
    a.lds_offb = P.rlds.offb_off;
    a.lds_pd = P.rlds.pd_off;
    a.lds_win = P.rlds.win_off;
    a.win_bytes = P.rlds.win_bytes;
    a.nbuf = 1;
    return a;
}

hipEvent_t take_event(smcx_lattice* h)
{
    if (!h->pool.empty()) {
        hipEvent_t e = h->pool.back();
        h->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int timed_launch(smcx_lattice* h, const void* kernel, dim3 grid, int block, size_t lds, hipStream_t st,
                 const SweepArgs& a)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (h->timing) {
        e0 = take_event(h);
        e1 = take_event(h);
        if (!e0 || !e1) return fail(SMCX_E_HIP, "hipEventCreate failed");
        SMCX_HIP(hipEventRecord(e0, st));
    }
    SMCX_HIP(launch_sweep(kernel, grid, block, lds, st, a));
    if (h->timing) {
        SMCX_HIP(hipEventRecord(e1, st));
        h->pending.emplace_back(e0, e1);
        ++h->timed_launches;
    }
    return SMCX_OK;
}

int pack_all(smcx_lattice* h, bool unpack, bool planar, hipStream_t st)
{
    const Plan& P = h->P;
    // natural rows to unpack, padded rows (halo rows included) to pack
    auto rows_of = [&](const Replica& R) {
        return unpack ? (int64_t)R.L[1] * R.L[2] : (int64_t)R.prows * (R.L[2] + 2 * kHalo);
    };
    const RepDev* reps = (const RepDev*)(h->ws + P.off_reps);
    if (P.R > 1 && P.R <= 65535) {
        // every replica in one launch (a ladder's replicas are small: one
        // launch each would cost more than their copies)
        int64_t most = 0;
        for (const Replica& R : P.reps) most = std::max(most, rows_of(R));
        SMCX_HIP(launch_pack(P.lattice, P.K, unpack, planar, h->occ, h->ws, reps, -1, most, P.R, st));
        return SMCX_OK;
    }
    for (int r = 0; r < P.R; ++r)
        SMCX_HIP(launch_pack(P.lattice, P.K, unpack, planar, h->occ, h->ws, reps, r, rows_of(P.reps[r]), 1, st));
    return SMCX_OK;
}

// The handle that currently owns each device's static workspace (a later
// smcx_lattice_init_static on the same device takes it over).
std::mutex g_static_mu;
const smcx_lattice* g_static_owner[kMaxDevices] = {};

int check_handle(const smcx_lattice* h)
{
    if (!h) return fail(SMCX_E_INVALID_ARG, "handle is NULL");
    if (h->static_dev >= 0) {
        std::lock_guard<std::mutex> lock(g_static_mu);
        if (g_static_owner[h->static_dev] != h)
            return fail(SMCX_E_INVALID_ARG,
                        "the static workspace of this handle's device was taken over by a later "
                        "smcx_lattice_init_static; this handle is no longer usable");
    }
    return SMCX_OK;
}

}  // namespace

extern "C" {

int smcx_version(void) { return SMCX_VERSION; }

const char* smcx_last_error(void) { return g_err.c_str(); }

int smcx_min_cell_edge(int32_t lattice, int32_t n_shells)
{
    if (lattice != SMCX_BCC && lattice != SMCX_FCC) return fail(SMCX_E_INVALID_ARG, "bad lattice");
    if (n_shells < 1 || n_shells > kMaxShells) return fail(SMCX_E_INVALID_ARG, "bad n_shells");
    return min_edge(lattice, n_shells);
}

int smcx_workspace_size(const smcx_desc* desc, size_t* bytes)
{
    if (!bytes) return fail(SMCX_E_INVALID_ARG, "bytes is NULL");
    Plan P;
    const int rc = make_plan(desc, P);
    if (rc != SMCX_OK) return rc;
    *bytes = P.total;
    return SMCX_OK;
}

int smcx_lattice_init(smcx_lattice** out, const smcx_desc* desc, uint8_t* occ_dev, void* ws_dev, size_t ws_bytes,
                      void* stream)
{
    if (!out) return fail(SMCX_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!occ_dev || !ws_dev) return fail(SMCX_E_INVALID_ARG, "occ_dev and ws_dev must be device pointers");
    if (((uintptr_t)ws_dev & 255) != 0) return fail(SMCX_E_INVALID_ARG, "workspace must be 256-byte aligned");
    smcx_lattice* h = new (std::nothrow) smcx_lattice();
    if (!h) return fail(SMCX_E_INVALID_ARG, "out of host memory");
    int rc = make_plan(desc, h->P);
    if (rc != SMCX_OK) {
        delete h;
        return rc;
    }
    const Plan& P = h->P;
    if (ws_bytes < P.total) {
        delete h;
        return fail(SMCX_E_WORKSPACE, "workspace too small: need " + std::to_string(P.total) + " bytes");
    }
    h->occ = occ_dev;
    h->ws = (uint8_t*)ws_dev;
    h->ws_bytes = ws_bytes;
    hipStream_t st = (hipStream_t)stream;

    // host images of the device tables
    std::vector<RepDev> reps(P.R);
    std::vector<int32_t> origins;
    std::vector<int64_t> tile_off(P.R + 1, 0);
    for (int r = 0; r < P.R; ++r) {
        const Replica& R = P.reps[r];
        RepDev& D = reps[r];
        std::memset(&D, 0, sizeof(D));
        for (int a = 0; a < 3; ++a) {
            D.L[a] = R.L[a];
            D.nc[a] = (int)R.edges[a].size();
            D.M[a] = R.M[a];
            D.emin[a] = *std::min_element(R.edges[a].begin(), R.edges[a].end());
            D.ntile[a] = R.ntile[a];
        }
        D.nA = R.nA;
        D.cs_off = (int)origins.size();
        for (int a = 0; a < 3; ++a) origins.insert(origins.end(), R.origin[a].begin(), R.origin[a].end());
        D.prow = R.prow;
        D.prows = R.prows;
        D.cp = R.cp;
        D.prowp = R.prowp;
        D.pad_off = R.pad_off;
        D.occ_off = R.occ_off;
        D.N = R.N;
        D.ntiles = R.ntiles;
        D.alias = 0;
        for (int s = 0; s < kMaxShells; ++s)
            for (int k = 0; k < kMaxZ1; ++k) {
                D.mult[s][k] = (uint8_t)R.mult[s][k];
                if (k < P.Z1 && R.mult[s][k] != (s == 0 ? 1 : 0)) D.alias = 1;
            }
        tile_off[r + 1] = tile_off[r] + R.ntiles;
    }
    const Geometry& G = kGeom[P.lattice];
    std::vector<int16_t> offP((size_t)P.m * P.Z1 * P.sumZ), offP_r(offP.size());
    std::vector<int32_t> offB((size_t)P.m * P.Z1), offB_r(offB.size());
    std::vector<int8_t> pd((size_t)4 * P.m * P.Z1);
    for (int b = 0; b < P.m; ++b)
        for (int k = 0; k < P.Z1; ++k) {
            const int* d1 = G.v[0][k];
            offB[b * P.Z1 + k] = lds_offset(P, P.LP, P.WY, b, d1[0], d1[1], d1[2]);
            if (P.rows) offB_r[b * P.Z1 + k] = lds_offset_planar(P, P.rLP, P.rWY, P.reps[0].cp, b, d1[0], d1[1], d1[2]);
            const Nb nb = nb_of(G, b, d1[0], d1[1], d1[2]);
            int8_t* q = &pd[(b * P.Z1 + k) * 4];
            q[0] = (int8_t)nb.dx; q[1] = (int8_t)nb.dy; q[2] = (int8_t)nb.dz; q[3] = (int8_t)nb.bt;
            int j = 0;
            for (int s = 0; s < P.S; ++s)
                for (int n = 0; n < G.Z[s]; ++n, ++j) {
                    const int vx = d1[0] + G.v[s][n][0], vy = d1[1] + G.v[s][n][1], vz = d1[2] + G.v[s][n][2];
                    offP[(b * P.Z1 + k) * P.sumZ + j] = (int16_t)lds_offset(P, P.LP, P.WY, b, vx, vy, vz);
                    if (P.rows)
                        offP_r[(b * P.Z1 + k) * P.sumZ + j] =
                            (int16_t)lds_offset_planar(P, P.rLP, P.rWY, P.reps[0].cp, b, vx, vy, vz);
                }
        }
    std::vector<int64_t> row_off(P.R + 1, 0);
    for (int r = 0; r < P.R; ++r) {
        reps[r].rg[0] = P.rows ? P.reps[r].rg[0] : 0;
        reps[r].rg[1] = P.rows ? P.reps[r].rg[1] : 0;
        row_off[r + 1] = row_off[r] + (int64_t)reps[r].rg[0] * reps[r].rg[1];
    }
    SMCX_HIP(hipMemcpyAsync(h->ws + P.off_reps, reps.data(), sizeof(RepDev) * P.R, hipMemcpyHostToDevice, st));
    SMCX_HIP(hipMemcpyAsync(h->ws + P.off_origins, origins.data(), sizeof(int32_t) * origins.size(), hipMemcpyHostToDevice, st));
    SMCX_HIP(hipMemcpyAsync(h->ws + P.off_tileoff, tile_off.data(), sizeof(int64_t) * tile_off.size(), hipMemcpyHostToDevice, st));
    SMCX_HIP(hipMemcpyAsync(h->ws + P.off_offP, offP.data(), sizeof(int16_t) * offP.size(), hipMemcpyHostToDevice, st));
    SMCX_HIP(hipMemcpyAsync(h->ws + P.off_offB, offB.data(), sizeof(int32_t) * offB.size(), hipMemcpyHostToDevice, st));
    SMCX_HIP(hipMemcpyAsync(h->ws + P.off_pd, pd.data(), pd.size(), hipMemcpyHostToDevice, st));
    SMCX_HIP(hipMemcpyAsync(h->ws + P.off_rowoff, row_off.data(), sizeof(int64_t) * row_off.size(), hipMemcpyHostToDevice, st));
    SMCX_HIP(hipMemcpyAsync(h->ws + P.off_offP_r, offP_r.data(), sizeof(int16_t) * offP_r.size(), hipMemcpyHostToDevice, st));
    SMCX_HIP(hipMemcpyAsync(h->ws + P.off_offB_r, offB_r.data(), sizeof(int32_t) * offB_r.size(), hipMemcpyHostToDevice, st));
    {
        // qSRO tables.  Neighbours of a basis-b site, shells in order; the
        // affected set of a swap of a basis-B site with its partner k: the
        // half-unit displacements 0, D_1[k], D_s[n] and D_1[k] + D_s[n],
        // without duplicates, in lexicographic (x, y, z) order (the order in
        // which a trial adds up the local-energy changes).
        const Geometry& G = kGeom[P.lattice];
        auto pack = [&](int b, int vx, int vy, int vz) {
            const Nb nb = nb_of(G, b, vx, vy, vz);
            return (int32_t)((nb.dx + 8) | (nb.dy + 8) << 8 | (nb.dz + 8) << 16 | nb.bt << 24);
        };
        std::vector<int32_t> qnbr((size_t)P.m * P.sumZ), qaff((size_t)P.m * P.Z1 * (1 + kQsroMaxAff), 0);
        for (int b = 0; b < P.m; ++b) {
            int j = 0;
            for (int sh = 0; sh < P.S; ++sh)
                for (int n = 0; n < G.Z[sh]; ++n) qnbr[(size_t)b * P.sumZ + j++] = pack(b, G.v[sh][n][0], G.v[sh][n][1], G.v[sh][n][2]);
        }
        int largest = 0;
        for (int b = 0; b < P.m; ++b)
            for (int k = 0; k < P.Z1; ++k) {
                std::vector<std::array<int, 3>> v;
                auto add = [&](int x, int y, int z) {
                    const std::array<int, 3> d{x, y, z};
                    if (std::find(v.begin(), v.end(), d) == v.end()) v.push_back(d);
                };
                const int* ab = G.v[0][k];
                add(0, 0, 0);
                add(ab[0], ab[1], ab[2]);
                for (int sh = 0; sh < P.S; ++sh)
                    for (int n = 0; n < G.Z[sh]; ++n) {
                        const int* d = G.v[sh][n];
                        add(d[0], d[1], d[2]);
                        add(ab[0] + d[0], ab[1] + d[1], ab[2] + d[2]);
                    }
                std::sort(v.begin(), v.end());
                if ((int)v.size() > kQsroMaxAff) return fail(SMCX_E_UNSUPPORTED, "qSRO affected set too large");
                int32_t* row = qaff.data() + (size_t)(b * P.Z1 + k) * (1 + kQsroMaxAff);
                row[0] = (int32_t)v.size();
                for (size_t i = 0; i < v.size(); ++i) row[1 + i] = pack(b, v[i][0], v[i][1], v[i][2]);
                largest = std::max(largest, (int)v.size());
            }
        h->P.qnaff = largest;
        // reach of a trial in cells: the farthest affected site plus the
        // farthest neighbour, per axis
        int ra = 0, rn = 0;
        for (int b = 0; b < P.m; ++b) {
            for (int k = 0; k < P.Z1; ++k) {
                const int32_t* row = qaff.data() + (size_t)(b * P.Z1 + k) * (1 + kQsroMaxAff);
                for (int i = 0; i < row[0]; ++i)
                    for (int sh = 0; sh < 3; ++sh) ra = std::max(ra, std::abs(((row[1 + i] >> (8 * sh)) & 0xff) - 8));
            }
            for (int j = 0; j < P.sumZ; ++j)
                for (int sh = 0; sh < 3; ++sh)
                    rn = std::max(rn, std::abs(((qnbr[(size_t)b * P.sumZ + j] >> (8 * sh)) & 0xff) - 8));
        }
        h->P.qreach = ra + rn;
        int32_t Zs[kMaxShells] = {0, 0, 0, 0};
        for (int sh = 0; sh < P.S; ++sh) Zs[sh] = G.Z[sh];
        SMCX_HIP(hipMemcpyAsync(h->ws + P.off_qnbr, qnbr.data(), sizeof(int32_t) * qnbr.size(), hipMemcpyHostToDevice, st));
        SMCX_HIP(hipMemcpyAsync(h->ws + P.off_qaff, qaff.data(), sizeof(int32_t) * qaff.size(), hipMemcpyHostToDevice, st));
        SMCX_HIP(hipMemcpyAsync(h->ws + P.off_qZ, Zs, sizeof(Zs), hipMemcpyHostToDevice, st));
        SMCX_HIP(hipStreamSynchronize(st));  // the host tables go out of scope
    }
    int32_t* bad = (int32_t*)(h->ws + P.off_misc);
    SMCX_HIP(launch_fill_i32(bad, 1, 0, st));
    SMCX_HIP(launch_validate(occ_dev, P.total_sites, P.K, bad, st));
    int32_t bad_h = 0;
    SMCX_HIP(hipMemcpyAsync(&bad_h, bad, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    SMCX_HIP(hipStreamSynchronize(st));
    if (bad_h) {
        delete h;
        return fail(SMCX_E_INVALID_ARG, "occupancy holds a species >= n_species");
    }
    h->k_stream = sweep_kernel(P.lattice, P.K, false, P.preset, P.nbuf);
    h->k_persistent = sweep_kernel(P.lattice, P.K, true, -1, 1);
    if (!h->k_stream || !h->k_persistent) {
        delete h;
        return fail(SMCX_E_UNSUPPORTED, "no sweep kernel for this configuration");
    }
    SMCX_HIP(set_sweep_lds_limit(h->k_stream, P.lds.total));
    SMCX_HIP(set_sweep_lds_limit(h->k_persistent, P.lds.total));
    // stream grid: every CU filled to the occupancy the LDS footprint allows
    int dev = 0, cus = 256, per_cu = 1;
    SMCX_HIP(hipGetDevice(&dev));
    SMCX_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    SMCX_HIP(sweep_occupancy(h->k_stream, P.block, P.lds.total, &per_cu));
    h->stream_wgs = 8 * std::max(1, (cus / 8) * std::max(1, per_cu));
    if (P.rows) {
        h->k_rows = row_kernel(P.lattice, P.K, P.S, P.rblock, P.row_preset);
        SMCX_HIP(set_sweep_lds_limit(h->k_rows, P.rlds.total));
        int rcu = 1;
        SMCX_HIP(sweep_occupancy(h->k_rows, P.rblock, P.rlds.total, &rcu));
        h->rows_wgs = 8 * std::max(1, (cus / 8) * std::max(1, rcu));
    }
    *out = h;
    g_err.clear();
    return SMCX_OK;
}

int smcx_lattice_init_static(smcx_lattice** out, const smcx_desc* desc, uint8_t* occ_dev, void* stream)
{
    if (!out) return fail(SMCX_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    size_t need = 0;
    if (int rc = smcx_workspace_size(desc, &need)) return rc;
    if (need > kStaticWorkspaceBytes)
        return fail(SMCX_E_WORKSPACE, "this description needs " + std::to_string(need) +
                                          " bytes of workspace; the static workspace holds " +
                                          std::to_string(kStaticWorkspaceBytes) +
                                          " (pass a workspace to smcx_lattice_init instead)");
    int dev = 0;
    SMCX_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SMCX_E_UNSUPPORTED, "device ordinal beyond the static workspaces");
    void* ws = nullptr;
    SMCX_HIP(static_workspace(&ws));
    {
        // the tables below overwrite the workspace: an earlier handle on this
        // device is unusable from here on
        std::lock_guard<std::mutex> lock(g_static_mu);
        g_static_owner[dev] = nullptr;
    }
    const int rc = smcx_lattice_init(out, desc, occ_dev, ws, kStaticWorkspaceBytes, stream);
    if (rc != SMCX_OK) return rc;
    (*out)->static_dev = dev;
    std::lock_guard<std::mutex> lock(g_static_mu);
    g_static_owner[dev] = *out;
    return SMCX_OK;
}

int smcx_lattice_destroy(smcx_lattice* h)
{
    if (!h) return SMCX_OK;
    if (h->static_dev >= 0) {
        std::lock_guard<std::mutex> lock(g_static_mu);
        if (g_static_owner[h->static_dev] == h) g_static_owner[h->static_dev] = nullptr;
    }
    for (auto& pr : h->pending) {
        (void)hipEventDestroy(pr.first);  // teardown: nothing to report to
        (void)hipEventDestroy(pr.second);
    }
    for (hipEvent_t e : h->pool) (void)hipEventDestroy(e);
    delete h;
    return SMCX_OK;
}

int smcx_get_schedule(const smcx_lattice* h, int32_t replica, int32_t* ncell_out, int32_t* cells_out,
                      int32_t* n_ministeps)
{
    if (int rc = check_handle(h)) return rc;
    if (replica < 0 || replica >= h->P.R) return fail(SMCX_E_INVALID_ARG, "replica out of range");
    const Replica& R = h->P.reps[replica];
    int pos = 0;
    for (int a = 0; a < 3; ++a) {
        if (ncell_out) ncell_out[a] = (int32_t)R.edges[a].size();
        for (int e : R.edges[a]) {
            if (cells_out) cells_out[pos] = e;
            ++pos;
        }
    }
    if (n_ministeps) *n_ministeps = R.nA;
    return SMCX_OK;
}

int smcx_set_epi(smcx_lattice* h, const double* V, void* stream)
{
    if (int rc = check_handle(h)) return rc;
    if (!V) return fail(SMCX_E_INVALID_ARG, "V is NULL");
    const Plan& P = h->P;
    const int K = P.K, S = P.S;
    for (int s = 0; s < S; ++s)
        for (int k = 0; k < K; ++k)
            for (int l = 0; l < K; ++l) {
                const double a = V[(s * K + k) * K + l], b = V[(s * K + l) * K + k];
                if (!(a == b)) return fail(SMCX_E_INVALID_ARG, "V must be symmetric in its species indices (and finite)");
            }
    h->V.assign(V, V + (size_t)S * K * K);
    h->Dhost.resize((size_t)K * K * S * K);
    for (int p = 0; p < K; ++p)
        for (int q = 0; q < K; ++q)
            for (int s = 0; s < S; ++s)
                for (int t = 0; t < K; ++t)
                    h->Dhost[((s * K + t) * K + p) * K + q] = V[(s * K + q) * K + t] - V[(s * K + p) * K + t];
    // Integer screen of dE (the kernels' first test): every D rounded to a
    // multiple of 2^-k, the largest k with all |D| 2^k below 2^23 (24-bit
    // signed operands), plus for each (p, q) the sum of half * those integers
    // (the counters' field bias), modulo 2^32.  A trial's integer sum is then
    // within sum_t |c_t| 2^-(k+1) <= (sum_s Z_s) 2^-k of sum c D, which is
    // within a few ulps of the binary64 dE; qeps bounds both.
    {
        double maxD = 0.0;
        for (double v : h->Dhost) maxD = std::max(maxD, std::fabs(v));
        int kq = 0;
        if (maxD > 0.0) {
            kq = (int)std::floor(std::log2(8388607.0 / maxD));
            while (std::ldexp(maxD, kq) > 8388607.0) --kq;
            kq = std::max(-100, std::min(100, kq));
        }
        const int half = K == 5 ? 32 : 128;
        const size_t nD = h->Dhost.size();
        h->Qhost.assign((size_t)qtab_entries(K, S) + 2, 0);
        for (size_t i = 0; i < nD; ++i) h->Qhost[i] = (int32_t)std::nearbyint(std::ldexp(h->Dhost[i], kq));
        for (int p = 0; p < K; ++p)
            for (int q = 0; q < K; ++q) {
                int64_t b = 0;
                for (int s = 0; s < S; ++s)
                    for (int t = 0; t < K; ++t) b += (int64_t)half * h->Qhost[((s * K + t) * K + p) * K + q];
                h->Qhost[nD + p * K + q] = (int32_t)(uint32_t)(uint64_t)b;
            }
        int sumZ = 0;
        for (int s = 0; s < S; ++s) sumZ += kGeom[P.lattice].Z[s];
        const float qscale = (float)std::ldexp(1.0, -kq);
        const float qeps = (float)((sumZ * std::ldexp(1.0, -kq) + 1e-12 * (1.0 + 64.0 * maxD)) * 1.001);
        std::memcpy(&h->Qhost[(size_t)qtab_entries(K, S)], &qscale, 4);
        std::memcpy(&h->Qhost[(size_t)qtab_entries(K, S) + 1], &qeps, 4);
    }
    hipStream_t st = (hipStream_t)stream;
    SMCX_HIP(hipMemcpyAsync(h->ws + P.off_D, h->Dhost.data(), sizeof(double) * h->Dhost.size(), hipMemcpyHostToDevice, st));
    SMCX_HIP(hipMemcpyAsync(h->ws + P.off_Q, h->Qhost.data(), sizeof(int32_t) * h->Qhost.size(), hipMemcpyHostToDevice, st));
    SMCX_HIP(hipMemcpyAsync(h->ws + P.off_V, h->V.data(), sizeof(double) * h->V.size(), hipMemcpyHostToDevice, st));
    SMCX_HIP(hipStreamSynchronize(st));
    h->epi_set = true;
    return SMCX_OK;
}

int smcx_set_qsro(smcx_lattice* h, const double* V, const double* W, void* stream)
{
    if (int rc = check_handle(h)) return rc;
    if (!V || !W) return fail(SMCX_E_INVALID_ARG, "V and W are required");
    const Plan& P = h->P;
    const int K = P.K, S = P.S;
    for (int s = 0; s < S; ++s)
        for (int k = 0; k < K; ++k) {
            if (!std::isfinite(W[s * K + k])) return fail(SMCX_E_INVALID_ARG, "W must be finite");
            for (int l = 0; l < K; ++l) {
                const double a = V[(s * K + k) * K + l], b = V[(s * K + l) * K + k];
                if (!(a == b)) return fail(SMCX_E_INVALID_ARG, "V must be symmetric in its species indices (and finite)");
            }
        }
    hipStream_t st = (hipStream_t)stream;
    SMCX_HIP(hipMemcpyAsync(h->ws + P.off_qV, V, sizeof(double) * S * K * K, hipMemcpyHostToDevice, st));
    SMCX_HIP(hipMemcpyAsync(h->ws + P.off_qW, W, sizeof(double) * S * K, hipMemcpyHostToDevice, st));
    SMCX_HIP(hipStreamSynchronize(st));
    h->qsro_set = true;
    return SMCX_OK;
}

int smcx_sweep_qsro(smcx_lattice* h, int32_t n_sweeps, uint64_t seed, uint32_t first_sweep, const double* beta_host,
                    int64_t* stats_dev, smcx_tie* ties_dev, int32_t tie_cap, int32_t* tie_count_dev, void* stream)
{
    if (int rc = check_handle(h)) return rc;
    if (!h->qsro_set) return fail(SMCX_E_NOT_READY, "smcx_set_qsro has not been called");
    if (n_sweeps < 0) return fail(SMCX_E_INVALID_ARG, "n_sweeps must be >= 0");
    if (n_sweeps > 0 && !beta_host) return fail(SMCX_E_INVALID_ARG, "beta_host is required");
    if (!stats_dev || !tie_count_dev) return fail(SMCX_E_INVALID_ARG, "stats and tie_count are required");
    if (tie_cap < 0 || (tie_cap > 0 && !ties_dev)) return fail(SMCX_E_INVALID_ARG, "ties_dev required when tie_cap > 0");
    const Plan& P = h->P;
    const Geometry& G = kGeom[P.lattice];
    // reach: largest |component| (half units) of the S shells' vectors
    int c = 0;
    for (int s = 0; s < P.S; ++s)
        for (int n = 0; n < G.Z[s]; ++n)
            for (int a = 0; a < 3; ++a) c = std::max(c, std::abs(G.v[s][n][a]));
    int ell = 1;
    while (!(2 * ell > 2 + 2 * c)) ++ell;  // interaction-zone rule
    for (const Replica& R : P.reps) {
        if (R.N > 0x7fffffffLL) return fail(SMCX_E_UNSUPPORTED, "qSRO sweeps need fewer than 2^31 sites per replica");
        for (int a = 0; a < 3; ++a) {
            if (R.L[a] <= c + 1) return fail(SMCX_E_INVALID_ARG, "qSRO needs every edge above the shells' reach + 1");
            if (R.edges[a].size() > 1)
                for (int e : R.edges[a])
                    if (e < ell)
                        return fail(SMCX_E_INVALID_ARG, "qSRO needs link cells of edge >= " + std::to_string(ell) +
                                                            " (interaction-zone rule); pass ell or cells accordingly");
        }
    }
    hipStream_t st = (hipStream_t)stream;
    const int32_t* origins = (const int32_t*)(h->ws + P.off_origins);
    std::vector<int> cs_off(P.R, 0);  // each replica's cell origins: nc + 1 entries per axis
    for (int r = 1; r < P.R; ++r) {
        const Replica& Q = P.reps[r - 1];
        cs_off[r] = cs_off[r - 1] + (int)(Q.origin[0].size() + Q.origin[1].size() + Q.origin[2].size());
    }
    for (int js = 0; js < n_sweeps; ++js)
        for (int r = 0; r < P.R; ++r) {
            const Replica& R = P.reps[r];
            QsroArgs A{};
            A.occ = h->occ + R.occ_off;
            A.L0 = R.L[0]; A.L1 = R.L[1]; A.L2 = R.L[2];
            A.K = P.K; A.S = P.S; A.Z1 = P.Z1; A.sumZ = P.sumZ; A.naff_max = kQsroMaxAff;
            A.ncx = (int)R.edges[0].size(); A.ncy = (int)R.edges[1].size(); A.ncz = (int)R.edges[2].size();
            A.reach = P.qreach;
            A.org = origins + cs_off[r];
            A.sweep = first_sweep + (uint32_t)js;
            A.replica = (uint32_t)r;
            A.seed = seed;
            A.beta = beta_host[(int64_t)js * P.R + r];
            A.aff = (const int32_t*)(h->ws + P.off_qaff);
            A.nbr = (const int32_t*)(h->ws + P.off_qnbr);
            A.V = (const double*)(h->ws + P.off_qV);
            A.W = (const double*)(h->ws + P.off_qW);
            A.Z = (const int32_t*)(h->ws + P.off_qZ);
            A.slots = (int64_t*)(h->ws + P.off_qslots);
            A.ties = ties_dev;
            A.tie_cap = tie_cap;
            A.tie_count = tie_count_dev;
            const int ncell = A.ncx * A.ncy * A.ncz;
            const int grid = std::min(ncell, kQsroGrid);
            SMCX_HIP(launch_fill_i64(A.slots, 3 * (int64_t)grid, 0, st));
            for (int tau = 0; tau < R.nA; ++tau) {
                A.b = tau % P.m;
                const int rest = tau / P.m;
                A.o0 = rest % R.M[0];
                A.o1 = (rest / R.M[0]) % R.M[1];
                A.o2 = rest / (R.M[0] * R.M[1]);
                SMCX_HIP(launch_qsro_ministep(P.lattice, A, grid, st));
            }
            SMCX_HIP(launch_qsro_reduce(A.slots, grid, stats_dev + 3 * (int64_t)r, st));
        }
    return SMCX_OK;
}

static int check_sweep_args(smcx_lattice* h, const double* beta_dev, int64_t* stats_dev, smcx_tie* ties_dev,
                            int32_t tie_cap, int32_t* tie_count_dev, int32_t mode)
{
    if (int rc = check_handle(h)) return rc;
    if (!h->epi_set) return fail(SMCX_E_NOT_READY, "smcx_set_epi has not been called");
    if (!beta_dev || !stats_dev || !tie_count_dev) return fail(SMCX_E_INVALID_ARG, "beta, stats and tie_count are required");
    if (tie_cap < 0 || (tie_cap > 0 && !ties_dev)) return fail(SMCX_E_INVALID_ARG, "ties_dev required when tie_cap > 0");
    if (mode < SMCX_MODE_AUTO || mode > SMCX_MODE_PLAIN) return fail(SMCX_E_INVALID_ARG, "bad mode");
    return SMCX_OK;
}

// Sweeps first_sweep .. first_sweep + n_sweeps - 1, mini-steps [tau_begin,
// tau_end) of each; beta_dev row js (R entries) belongs to sweep js.
static int run_sweeps(smcx_lattice* h, int32_t n_sweeps, uint64_t seed, uint32_t first_sweep, int tau_begin,
                      int tau_end, const double* beta_dev, int64_t* stats_dev, smcx_tie* ties_dev, int32_t tie_cap,
                      int32_t* tie_count_dev, int32_t mode, hipStream_t st, uint32_t* sweep_counter = nullptr,
                      int64_t beta_row_stride = -1)
{
    // sweep js reads beta row js (R entries) by default; a stride of 0 gives
    // every sweep of the call the same row
    const int64_t bstride = beta_row_stride < 0 ? (int64_t)h->P.R : beta_row_stride;
    // with a device sweep counter (graph capture) the kernels read the sweep
    // index from it and first_sweep counts from 0
    if (sweep_counter) first_sweep = 0;
    const Plan& P = h->P;
    // auto: one persistent launch for lattices too small to fill a launch per
    // mini-step group; row windows where they apply (the ladder of 256 BCC
    // replicas runs 10x faster in row launches than in one workgroup per
    // replica); otherwise persistent for several replicas
    if (mode == SMCX_MODE_AUTO)
        mode = P.total_sites <= (1 << 16) ? SMCX_MODE_PERSISTENT
                                          : (P.rows || P.R == 1 ? SMCX_MODE_STREAM : SMCX_MODE_PERSISTENT);
    // the row kernel reads basis-planar rows; replicas of different
    // decompositions share its launches only over whole sweeps
    const bool rows = mode == SMCX_MODE_STREAM && P.rows && (!P.rows_mixed || (tau_begin == 0 && tau_end >= P.max_nA));
    const bool planar = rows;
    if (int rc = pack_all(h, false, planar, st)) return rc;
    SweepArgs a = base_args(h);
    a.seed = seed;
    a.stats = stats_dev;
    a.ties = ties_dev;
    a.tie_cap = tie_cap;
    a.tie_count = tie_count_dev;
    a.n_sweeps = n_sweeps;
    a.tau_begin = tau_begin;
    a.tau_end = tau_end;
    a.sweep_counter = sweep_counter;
    // one launch per group of mini-steps that share an offset (and a window)
    auto group_end = [&](int g, int end) { return std::min(end, (g / P.group + 1) * P.group); };
    if (mode == SMCX_MODE_PERSISTENT) {
        a.first_sweep = first_sweep;
        a.beta = beta_dev;
        a.beta_stride = bstride;
        a.nb = P.group;
        if (int rc = timed_launch(h, h->k_persistent, dim3(P.R), P.block, P.lds.total, st, a)) return rc;
    } else if (rows) {
        // one launch per (o_y, o_z) group: every o_x and basis site
        SweepArgs ra = row_args(h);
        ra.seed = a.seed;
        ra.stats = a.stats;
        ra.ties = a.ties;
        ra.tie_cap = a.tie_cap;
        ra.tie_count = a.tie_count;
        ra.sweep_counter = sweep_counter;
        const int G = P.m * P.reps[0].M[0];
        const dim3 grid((unsigned)std::min<int64_t>(h->rows_wgs, 8 * ((P.total_rowgroups + 7) / 8)));
        int max_groups = 0;
        for (const Replica& R : P.reps) max_groups = std::max(max_groups, R.M[1] * R.M[2]);
        for (int js = 0; js < n_sweeps; ++js) {
            ra.first_sweep = first_sweep + (uint32_t)js;
            ra.beta = beta_dev + (int64_t)js * bstride;
            if (P.rows_mixed) {
                for (int q = 0; q < max_groups; ++q) {
                    ra.gq = q;
                    if (int rc = timed_launch(h, h->k_rows, grid, P.rblock, P.rlds.total, st, ra)) return rc;
                }
                continue;
            }
            const int end = std::min(tau_end, P.max_nA);
            for (int g = tau_begin; g < end;) {
                const int ge = std::min(end, (g / G + 1) * G);
                ra.g = g;
                ra.nb = ge - g;
                if (int rc = timed_launch(h, h->k_rows, grid, P.rblock, P.rlds.total, st, ra)) return rc;
                g = ge;
            }
        }
    } else if (mode == SMCX_MODE_STREAM) {
        const dim3 grid((unsigned)std::min<int64_t>(h->stream_wgs, 8 * ((P.total_tiles + 7) / 8)));
        for (int js = 0; js < n_sweeps; ++js) {
            a.first_sweep = first_sweep + (uint32_t)js;
            a.beta = beta_dev + (int64_t)js * bstride;
            const int end = std::min(tau_end, P.max_nA);
            for (int g = tau_begin; g < end; g = group_end(g, end)) {
                a.g = g;
                a.nb = group_end(g, end) - g;
                if (int rc = timed_launch(h, h->k_stream, grid, P.block, P.lds.total, st, a)) return rc;
            }
        }
    } else {
        for (int js = 0; js < n_sweeps; ++js) {
            a.first_sweep = first_sweep + (uint32_t)js;
            a.beta = beta_dev + (int64_t)js * bstride;
            for (int r = 0; r < P.R; ++r) {
                a.only_rep = r;
                const dim3 grid((unsigned)std::min<int64_t>(h->stream_wgs, 8 * ((P.reps[r].ntiles + 7) / 8)));
                const int end = std::min(tau_end, P.reps[r].nA);
                for (int g = tau_begin; g < end; g = group_end(g, end)) {
                    a.g = g;
                    a.nb = group_end(g, end) - g;
                    if (int rc = timed_launch(h, h->k_stream, grid, P.block, P.lds.total, st, a)) return rc;
                }
            }
        }
    }
    return pack_all(h, true, planar, st);
}

int smcx_sweep(smcx_lattice* h, int32_t n_sweeps, uint64_t seed, uint32_t first_sweep, const double* beta_dev,
               int64_t* stats_dev, smcx_tie* ties_dev, int32_t tie_cap, int32_t* tie_count_dev, int32_t mode,
               void* stream)
{
    if (n_sweeps < 0) return fail(SMCX_E_INVALID_ARG, "n_sweeps must be >= 0");
    if (int rc = check_sweep_args(h, beta_dev, stats_dev, ties_dev, tie_cap, tie_count_dev, mode)) return rc;
    if (n_sweeps == 0) return SMCX_OK;
    return run_sweeps(h, n_sweeps, seed, first_sweep, 0, h->P.max_nA, beta_dev, stats_dev, ties_dev, tie_cap,
                      tie_count_dev, mode, (hipStream_t)stream);
}

int smcx_sweep_partial(smcx_lattice* h, uint32_t sweep, int32_t tau_begin, int32_t tau_end, uint64_t seed,
                       const double* beta_dev, int64_t* stats_dev, smcx_tie* ties_dev, int32_t tie_cap,
                       int32_t* tie_count_dev, int32_t mode, void* stream)
{
    if (int rc = check_sweep_args(h, beta_dev, stats_dev, ties_dev, tie_cap, tie_count_dev, mode)) return rc;
    if (tau_begin < 0 || tau_end < tau_begin || tau_end > h->P.max_nA)
        return fail(SMCX_E_INVALID_ARG, "mini-step range out of bounds");
    if (tau_end == tau_begin) return SMCX_OK;
    return run_sweeps(h, 1, seed, sweep, tau_begin, tau_end, beta_dev, stats_dev, ties_dev, tie_cap, tie_count_dev,
                      mode, (hipStream_t)stream);
}

int smcx_pair_counts(smcx_lattice* h, int64_t* counts_dev, void* stream)
{
    if (int rc = check_handle(h)) return rc;
    if (!counts_dev) return fail(SMCX_E_INVALID_ARG, "counts_dev is NULL");
    const Plan& P = h->P;
    hipStream_t st = (hipStream_t)stream;
    const int64_t per = (int64_t)P.S * P.K * P.K;
    SMCX_HIP(launch_fill_i64(counts_dev, per * P.R, 0, st));
    // replicas of one size lie back to back: one batched launch
    bool one_size = P.R <= 65535;
    for (const Replica& R : P.reps)
        for (int a = 0; a < 3; ++a) one_size &= R.L[a] == P.reps[0].L[a];
    if (one_size) {
        const Replica& R = P.reps[0];
        SMCX_HIP(launch_pair_counts(P.lattice, P.K, P.S, h->occ, R.N, R.L, P.R, counts_dev, st));
        return SMCX_OK;
    }
    for (int r = 0; r < P.R; ++r) {
        const Replica& R = P.reps[r];
        SMCX_HIP(launch_pair_counts(P.lattice, P.K, P.S, h->occ + R.occ_off, R.N, R.L, 1, counts_dev + per * r, st));
    }
    return SMCX_OK;
}

static int fetch_counts(smcx_lattice* h, int64_t* counts_dev, hipStream_t st)
{
    const Plan& P = h->P;
    if (int rc = smcx_pair_counts(h, counts_dev, st)) return rc;
    h->counts_host.resize((size_t)P.R * P.S * P.K * P.K);
    SMCX_HIP(hipMemcpyAsync(h->counts_host.data(), counts_dev, sizeof(int64_t) * h->counts_host.size(),
                            hipMemcpyDeviceToHost, st));
    SMCX_HIP(hipStreamSynchronize(st));
    return SMCX_OK;
}

int smcx_energy(smcx_lattice* h, int64_t* counts_dev, double* E_host, void* stream)
{
    if (int rc = check_handle(h)) return rc;
    if (!h->epi_set) return fail(SMCX_E_NOT_READY, "smcx_set_epi has not been called");
    if (!E_host) return fail(SMCX_E_INVALID_ARG, "E_host is NULL");
    if (int rc = fetch_counts(h, counts_dev, (hipStream_t)stream)) return rc;
    const Plan& P = h->P;
    const int K = P.K, S = P.S;
    for (int r = 0; r < P.R; ++r) {
        const int64_t* C = h->counts_host.data() + (size_t)r * S * K * K;
        double acc = 0.0;
        for (int s = 0; s < S; ++s)
            for (int k = 0; k < K; ++k)
                for (int l = 0; l < K; ++l) {
                    const size_t i = ((size_t)s * K + k) * K + l;
                    acc = acc + (double)C[i] * h->V[i];
                }
        E_host[r] = 0.5 * acc;
    }
    return SMCX_OK;
}

int smcx_energy_dev(smcx_lattice* h, int64_t* counts_dev, double* E_dev, void* stream)
{
    if (int rc = check_handle(h)) return rc;
    if (!h->epi_set) return fail(SMCX_E_NOT_READY, "smcx_set_epi has not been called");
    if (!counts_dev || !E_dev) return fail(SMCX_E_INVALID_ARG, "counts_dev and E_dev are required");
    if (int rc = smcx_pair_counts(h, counts_dev, stream)) return rc;
    const Plan& P = h->P;
    SMCX_HIP(launch_energy(counts_dev, (const double*)(h->ws + P.off_V), P.R, P.S * P.K * P.K, E_dev,
                           (hipStream_t)stream));
    return SMCX_OK;
}

int smcx_exchange(smcx_lattice* h, int32_t round, uint64_t seed, const double* beta_slot_dev, int32_t* rep_at_dev,
                  double* beta_dev, int32_t n_beta_rows, int64_t* counts_dev, double* E_dev, int64_t* xstats_dev,
                  smcx_tie* ties_dev, int32_t tie_cap, int32_t* tie_count_dev, void* stream)
{
    if (int rc = check_handle(h)) return rc;
    if (!h->epi_set) return fail(SMCX_E_NOT_READY, "smcx_set_epi has not been called");
    if (round < 0) return fail(SMCX_E_INVALID_ARG, "round must be >= 0");
    if (!beta_slot_dev || !rep_at_dev || !counts_dev || !E_dev || !xstats_dev || !tie_count_dev)
        return fail(SMCX_E_INVALID_ARG, "beta_slot, rep_at, counts, E, xstats and tie_count are required");
    if (n_beta_rows < 0 || (n_beta_rows > 0 && !beta_dev))
        return fail(SMCX_E_INVALID_ARG, "beta_dev is required when n_beta_rows > 0");
    if (tie_cap < 0 || (tie_cap > 0 && !ties_dev)) return fail(SMCX_E_INVALID_ARG, "ties_dev required when tie_cap > 0");
    const Plan& P = h->P;
    for (const Replica& R : P.reps)
        for (int a = 0; a < 3; ++a)
            if (R.L[a] != P.reps[0].L[a])
                return fail(SMCX_E_INVALID_ARG, "replica exchange needs replicas of one size");
    if (int rc = smcx_energy_dev(h, counts_dev, E_dev, stream)) return rc;
    SMCX_HIP(launch_exchange(E_dev, beta_slot_dev, rep_at_dev, P.R, seed, (uint32_t)round, beta_dev, n_beta_rows,
                             xstats_dev, ties_dev, tie_cap, tie_count_dev, (hipStream_t)stream));
    return SMCX_OK;
}

int smcx_anneal(smcx_lattice* h, int32_t n_steps, int32_t warmup, int32_t record, uint64_t seed, uint32_t first_sweep,
                const double* beta_steps_dev, int64_t* counts_dev, double* E_dev, double* cv_dev, int64_t* stats_dev,
                smcx_tie* ties_dev, int32_t tie_cap, int32_t* tie_count_dev, int32_t mode, void* stream)
{
    if (n_steps < 0 || warmup < 0 || record < 0) return fail(SMCX_E_INVALID_ARG, "n_steps, warmup and record must be >= 0");
    if (int rc = check_sweep_args(h, beta_steps_dev, stats_dev, ties_dev, tie_cap, tie_count_dev, mode)) return rc;
    if (record > 0 && (!counts_dev || !E_dev || !cv_dev))
        return fail(SMCX_E_INVALID_ARG, "counts_dev, E_dev and cv_dev are required when record > 0");
    const Plan& P = h->P;
    hipStream_t st = (hipStream_t)stream;
    const int64_t per = (int64_t)warmup + record;
    if ((int64_t)first_sweep + per * n_steps > 0xffffffffLL) return fail(SMCX_E_INVALID_ARG, "sweep index overflows 32 bits");
    for (int s = 0; s < n_steps; ++s) {
        const double* b = beta_steps_dev + (int64_t)s * P.R;
        const uint32_t t0 = first_sweep + (uint32_t)(s * per);
        if (warmup > 0)
            if (int rc = run_sweeps(h, warmup, seed, t0, 0, P.max_nA, b, stats_dev, ties_dev, tie_cap, tie_count_dev,
                                    mode, st, nullptr, 0))
                return rc;
        for (int j = 0; j < record; ++j) {
            if (int rc = run_sweeps(h, 1, seed, t0 + (uint32_t)(warmup + j), 0, P.max_nA, b, stats_dev, ties_dev,
                                    tie_cap, tie_count_dev, mode, st, nullptr, 0))
                return rc;
            if (int rc = smcx_energy_dev(h, counts_dev, E_dev + ((int64_t)s * record + j) * P.R, stream)) return rc;
        }
    }
    if (record > 0 && n_steps > 0)
        SMCX_HIP(launch_heat_capacity(E_dev, beta_steps_dev, (const RepDev*)(h->ws + P.off_reps), n_steps, record, P.R,
                                      cv_dev, st));
    return SMCX_OK;
}

int smcx_local_energy(smcx_lattice* h, int32_t replica, double* e_dev, void* stream)
{
    if (int rc = check_handle(h)) return rc;
    if (!h->epi_set) return fail(SMCX_E_NOT_READY, "smcx_set_epi has not been called");
    const Plan& P = h->P;
    if (replica < 0 || replica >= P.R) return fail(SMCX_E_INVALID_ARG, "replica out of range");
    if (!e_dev) return fail(SMCX_E_INVALID_ARG, "e_dev is NULL");
    const Replica& R = P.reps[replica];
    if (R.N > 0x7fffffffLL) return fail(SMCX_E_UNSUPPORTED, "local energies need fewer than 2^31 sites per replica");
    SMCX_HIP(launch_local_energy(P.lattice, h->occ + R.occ_off, R.L, P.K, P.S, (const double*)(h->ws + P.off_V), e_dev,
                                 (hipStream_t)stream));
    return SMCX_OK;
}

int smcx_clusters(smcx_lattice* h, int32_t replica, const double* e_dev, double threshold, int32_t* label_dev,
                  int32_t* size_dev, int64_t* n_clusters_dev, void* stream)
{
    if (int rc = check_handle(h)) return rc;
    const Plan& P = h->P;
    if (replica < 0 || replica >= P.R) return fail(SMCX_E_INVALID_ARG, "replica out of range");
    if (!e_dev || !label_dev || !size_dev || !n_clusters_dev)
        return fail(SMCX_E_INVALID_ARG, "e_dev, label_dev, size_dev and n_clusters_dev are required");
    const Replica& R = P.reps[replica];
    if (R.N > 0x7fffffffLL) return fail(SMCX_E_UNSUPPORTED, "clusters need fewer than 2^31 sites per replica");
    SMCX_HIP(launch_clusters(P.lattice, e_dev, R.L, threshold, label_dev, size_dev, n_clusters_dev, (hipStream_t)stream));
    return SMCX_OK;
}

int smcx_sro(smcx_lattice* h, int64_t* counts_dev, double* alpha_host, void* stream)
{
    if (int rc = check_handle(h)) return rc;
    if (!alpha_host) return fail(SMCX_E_INVALID_ARG, "alpha_host is NULL");
    if (int rc = fetch_counts(h, counts_dev, (hipStream_t)stream)) return rc;
    const Plan& P = h->P;
    const int K = P.K, S = P.S;
    const Geometry& G = kGeom[P.lattice];
    for (int r = 0; r < P.R; ++r) {
        const int64_t* C = h->counts_host.data() + (size_t)r * S * K * K;
        int64_t Nk[kMaxK];
        int64_t N = 0;
        for (int k = 0; k < K; ++k) {
            int64_t row = 0;
            for (int l = 0; l < K; ++l) row += C[k * K + l];
            Nk[k] = row / G.Z[0];
            if (Nk[k] == 0) return fail(SMCX_E_INVALID_ARG, "species " + std::to_string(k) + " absent from replica " + std::to_string(r));
            N += Nk[k];
        }
        double* al = alpha_host + (size_t)r * S * K * K;
        for (int s = 0; s < S; ++s)
            for (int k = 0; k < K; ++k)
                for (int l = 0; l < K; ++l) {
                    const size_t i = ((size_t)s * K + k) * K + l;
                    al[i] = 1.0 - ((double)C[i] * (double)N) / (((double)G.Z[s] * (double)Nk[k]) * (double)Nk[l]);
                }
    }
    return SMCX_OK;
}

int smcx_energy_backward(int32_t lattice, const int32_t* dims, int32_t n_species, int32_t n_shells,
                         const uint8_t* occ_batch_dev, int32_t B, int64_t* counts_dev, void* stream)
{
    if (lattice != SMCX_BCC && lattice != SMCX_FCC) return fail(SMCX_E_INVALID_ARG, "bad lattice");
    if (n_species < 2 || n_species > kMaxK) return fail(SMCX_E_INVALID_ARG, "n_species must be in 2..8");
    if (n_shells < 1 || n_shells > kMaxShells) return fail(SMCX_E_INVALID_ARG, "n_shells must be in 1..4");
    if (!dims || B < 0) return fail(SMCX_E_INVALID_ARG, "bad dims or B");
    if (B == 0) return SMCX_OK;
    if (!occ_batch_dev || !counts_dev) return fail(SMCX_E_INVALID_ARG, "NULL device pointer");
    const Geometry& G = kGeom[lattice];
    for (int a = 0; a < 3; ++a)
        if (dims[a] < 2) return fail(SMCX_E_INVALID_ARG, "every dimension must be >= 2");
    for (int s = 0; s < n_shells; ++s)
        for (int n = 0; n < G.Z[s]; ++n) {
            bool self = true;
            for (int a = 0; a < 3; ++a) self &= (G.v[s][n][a] % (2 * dims[a])) == 0;
            if (self) return fail(SMCX_E_INVALID_ARG, "lattice too small: a site would be its own neighbour");
        }
    const int64_t N = (int64_t)lattice_m(lattice) * dims[0] * dims[1] * dims[2];
    hipStream_t st = (hipStream_t)stream;
    const int64_t per = (int64_t)n_shells * n_species * n_species;
    // species check: the flag lives in the first word of counts_dev, which
    // the counts overwrite afterwards (a species >= K would shift a counter
    // field out of range and silently miscount)
    {
        int32_t* bad = (int32_t*)counts_dev;
        SMCX_HIP(launch_fill_i32(bad, 1, 0, st));
        SMCX_HIP(launch_validate(occ_batch_dev, N * (int64_t)B, n_species, bad, st));
        int32_t bad_h = 0;
        SMCX_HIP(hipMemcpyAsync(&bad_h, bad, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        SMCX_HIP(hipStreamSynchronize(st));
        if (bad_h) return fail(SMCX_E_INVALID_ARG, "a configuration holds a species >= n_species");
    }
    SMCX_HIP(launch_fill_i64(counts_dev, per * B, 0, st));
    for (int32_t b0 = 0; b0 < B; b0 += 65535) {
        const int nb = std::min<int32_t>(65535, B - b0);
        SMCX_HIP(launch_pair_counts(lattice, n_species, n_shells, occ_batch_dev + (int64_t)b0 * N, N, dims, nb,
                                    counts_dev + per * b0, st));
    }
    return SMCX_OK;
}

int smcx_energy_of_counts(const int64_t* counts_dev, const double* V_dev, int32_t B, int32_t n_terms,
                          double* E_dev, void* stream)
{
    if (B < 0 || n_terms < 1) return fail(SMCX_E_INVALID_ARG, "B must be >= 0 and n_terms >= 1");
    if (B == 0) return SMCX_OK;
    if (!counts_dev || !V_dev || !E_dev) return fail(SMCX_E_INVALID_ARG, "NULL device pointer");
    SMCX_HIP(launch_energy(counts_dev, V_dev, B, n_terms, E_dev, (hipStream_t)stream));
    return SMCX_OK;
}

int smcx_energy_grad(const int64_t* counts_dev, const double* g_dev, int32_t B, int32_t n_terms, double* grad_dev,
                     void* stream)
{
    if (B < 0 || n_terms < 1) return fail(SMCX_E_INVALID_ARG, "B must be >= 0 and n_terms >= 1");
    if (!counts_dev && B > 0) return fail(SMCX_E_INVALID_ARG, "NULL device pointer");
    if (!g_dev && B > 0) return fail(SMCX_E_INVALID_ARG, "NULL device pointer");
    if (!grad_dev) return fail(SMCX_E_INVALID_ARG, "NULL device pointer");
    SMCX_HIP(launch_energy_grad(counts_dev, g_dev, B, n_terms, grad_dev, (hipStream_t)stream));
    return SMCX_OK;
}

int smcx_ladder_capture(smcx_lattice* h, int32_t n_sweeps, uint64_t seed, const double* beta_dev,
                        uint32_t* sweep_counter_dev, int64_t* stats_dev, smcx_tie* ties_dev, int32_t tie_cap,
                        int32_t* tie_count_dev, void* stream, void** graph_out)
{
    if (int rc = check_handle(h)) return rc;
    if (!graph_out) return fail(SMCX_E_INVALID_ARG, "graph_out is NULL");
    *graph_out = nullptr;
    if (!h->epi_set) return fail(SMCX_E_NOT_READY, "smcx_set_epi has not been called");
    if (n_sweeps < 1) return fail(SMCX_E_INVALID_ARG, "n_sweeps must be >= 1");
    if (!beta_dev || !sweep_counter_dev || !stats_dev || !tie_count_dev)
        return fail(SMCX_E_INVALID_ARG, "beta, sweep counter, stats and tie_count are required");
    if (tie_cap < 0 || (tie_cap > 0 && !ties_dev)) return fail(SMCX_E_INVALID_ARG, "ties_dev required when tie_cap > 0");
    if (h->timing) return fail(SMCX_E_INVALID_ARG, "disable timing before capturing a graph");
    if (stream == nullptr) return fail(SMCX_E_INVALID_ARG, "the legacy default stream cannot be captured; pass a created stream");
    const Plan& P = h->P;
    hipStream_t st = (hipStream_t)stream;
    SMCX_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    SweepArgs a = base_args(h);
    a.seed = seed;
    a.stats = stats_dev;
    a.ties = ties_dev;
    a.tie_cap = tie_cap;
    a.tie_count = tie_count_dev;
    a.n_sweeps = n_sweeps;
    a.first_sweep = 0;
    a.sweep_counter = sweep_counter_dev;
    a.beta = beta_dev;
    a.beta_stride = 0;
    a.tau_begin = 0;
    a.tau_end = P.max_nA;
    a.nb = P.group;
    int rc = pack_all(h, false, false, st);
    hipError_t e = hipSuccess;
    if (rc == SMCX_OK) e = launch_sweep(h->k_persistent, dim3(P.R), P.block, P.lds.total, st, a);
    if (rc == SMCX_OK && e == hipSuccess) e = launch_advance_counter(sweep_counter_dev, (uint32_t)n_sweeps, st);
    if (rc == SMCX_OK && e == hipSuccess) rc = pack_all(h, true, false, st);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(st, &graph);
    if (rc != SMCX_OK) {
        if (graph) (void)hipGraphDestroy(graph);  // the capture error is the one reported
        return rc;
    }
    if (e != hipSuccess || e2 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(SMCX_E_HIP, std::string("graph capture failed: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);  // the executable graph keeps what it needs
    if (e != hipSuccess) return fail(SMCX_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    *graph_out = (void*)exec;
    return SMCX_OK;
}

int smcx_sweep_capture(smcx_lattice* h, int32_t n_sweeps, uint64_t seed, const double* beta_dev,
                       uint32_t* sweep_counter_dev, int64_t* stats_dev, smcx_tie* ties_dev, int32_t tie_cap,
                       int32_t* tie_count_dev, int32_t mode, void* stream, void** graph_out)
{
    if (!graph_out) return fail(SMCX_E_INVALID_ARG, "graph_out is NULL");
    *graph_out = nullptr;
    if (n_sweeps < 1) return fail(SMCX_E_INVALID_ARG, "n_sweeps must be >= 1");
    if (int rc = check_sweep_args(h, beta_dev, stats_dev, ties_dev, tie_cap, tie_count_dev, mode)) return rc;
    if (!sweep_counter_dev) return fail(SMCX_E_INVALID_ARG, "sweep_counter_dev is NULL");
    if (h->timing) return fail(SMCX_E_INVALID_ARG, "disable timing before capturing a graph");
    if (stream == nullptr) return fail(SMCX_E_INVALID_ARG, "the legacy default stream cannot be captured; pass a created stream");
    hipStream_t st = (hipStream_t)stream;
    SMCX_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    int rc = run_sweeps(h, n_sweeps, seed, 0, 0, h->P.max_nA, beta_dev, stats_dev, ties_dev, tie_cap, tie_count_dev,
                        mode, st, sweep_counter_dev);
    hipError_t e = hipSuccess;
    if (rc == SMCX_OK) e = launch_advance_counter(sweep_counter_dev, (uint32_t)n_sweeps, st);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(st, &graph);
    if (rc != SMCX_OK) {
        if (graph) (void)hipGraphDestroy(graph);  // the capture error is the one reported
        return rc;
    }
    if (e != hipSuccess || e2 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(SMCX_E_HIP, std::string("graph capture failed: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);  // the executable graph keeps what it needs
    if (e != hipSuccess) return fail(SMCX_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    *graph_out = (void*)exec;
    return SMCX_OK;
}

int smcx_graph_launch(void* graph, void* stream)
{
    if (!graph) return fail(SMCX_E_INVALID_ARG, "graph is NULL");
    SMCX_HIP(hipGraphLaunch((hipGraphExec_t)graph, (hipStream_t)stream));
    return SMCX_OK;
}

int smcx_graph_destroy(void* graph)
{
    if (!graph) return SMCX_OK;
    SMCX_HIP(hipGraphExecDestroy((hipGraphExec_t)graph));
    return SMCX_OK;
}

int smcx_timing_enable(smcx_lattice* h, int32_t enable)
{
    if (int rc = check_handle(h)) return rc;
    h->timing = enable != 0;
    return SMCX_OK;
}

int smcx_timing_read(smcx_lattice* h, double* ms_out, int64_t* launches_out)
{
    if (int rc = check_handle(h)) return rc;
    double total = 0.0;
    if (!h->pending.empty()) SMCX_HIP(hipEventSynchronize(h->pending.back().second));
    for (auto& pr : h->pending) {
        float ms = 0.f;
        SMCX_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
        total += ms;
        h->pool.push_back(pr.first);
        h->pool.push_back(pr.second);
    }
    h->pending.clear();
    if (ms_out) *ms_out = total;
    if (launches_out) *launches_out = h->timed_launches;
    h->timed_launches = 0;
    return SMCX_OK;
}

}  // extern "C"
