// gfx950 kernels of libsmcx: link-cell parallel swap Metropolis sweeps with a
// multi-shell EPI energy, pair counting, and helpers.
//
// Trial (one lane per link cell of a tile):
//   1. Philox4x32-10 on counter (site, sweep, replica) gives the partner
//      direction k and the uniform u (Methods, "Random number generator"
//      bullet: one draw per trial);
//   2. the tile window around the active sites is staged from the padded
//      HBM copy into LDS with 16-byte loads, species stored pre-shifted
//      (8 * sigma) so that a neighbour costs one LDS byte read and one
//      shift-add into a packed per-shell counter (8 bits per species);
//   3. dE = sum_s sum_t (n_a - n_b)[s][t] * (V_s[q][t] - V_s[p][t]) in binary64
//      from the integer counters, s and t ascending, the a-b bond excluded
//      (Methods, "The EPI and qSRO model": the energy change of a pair model
//      is twice the change of the two local energies);
//   4. Metropolis test (Supplementary, acceptance equation), near-ties within
//      1e-12 logged; accepted swaps write two bytes (and their halo images)
//      straight to HBM.
// The trials of one mini-step are independent (Results, LIZ / LIZ+
// argument), so a mini-step is one grid-wide wave of independent lanes and
// mini-steps are ordered by launch order or by workgroup barriers.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <type_traits>

#include "smcx_internal.h"
#include "smcx_launch.h"

namespace smcx {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Ten rounds of the
// 4-word S-box: two 32x32->64 products of words 0 and 2 with the multipliers,
// high halves xored with words 1/3 and the round key, low halves kept; the
// key advances by the Weyl increments between rounds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t& o0,
                                              uint32_t& o1, uint32_t& o2, uint32_t& o3)
{
    // the key is wave-uniform: keep it in scalar registers and let the round
    // keys be formed here, not hoisted out of the trial loops as 20 live SGPRs
    asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        // round 0: words 1 and 3 are often wave-uniform, so their xor with
        // the key is left to scalar code; later rounds take one three-input
        // xor (truth table 0x96) instead of two xors
        const uint32_t n0 = r == 0 ? (uint32_t)(p1 >> 32) ^ (c1 ^ k0)
                                   : __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = r == 0 ? (uint32_t)(p0 >> 32) ^ (c3 ^ k1)
                                   : __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    o0 = c0; o1 = c1; o2 = c2; o3 = c3;
}

// Packed per-shell neighbour counters: F bits per species, one field per
// species, biased by `half` when two counters are subtracted so that every
// field of (n_a + bias - n_b) stays in [half - 24, half + 24] (a shell has at
// most 24 sites) and no borrow crosses fields.  Encoding 1: K <= 4, 8-bit
// fields in 32 bits; 3: K = 5, 6-bit fields in 32 bits; 2: K <= 8, 8-bit
// fields in 64 bits.  The padded copy and the LDS window hold F * species.
template <int E> struct Enc;
template <> struct Enc<1> {
    using T = uint32_t;
    static constexpr int F = 8, KP = 4, half = 128;
    static constexpr uint32_t bias = 0x80808080u, mask = 0xFF;
};
template <> struct Enc<3> {
    using T = uint32_t;
    static constexpr int F = 6, KP = 5, half = 32;
    static constexpr uint32_t bias = 32u | 32u << 6 | 32u << 12 | 32u << 18 | 32u << 24, mask = 0x3F;
};
template <> struct Enc<2> {
    using T = uint64_t;
    static constexpr int F = 8, KP = 8, half = 128;
    static constexpr uint64_t bias = 0x8080808080808080ull, mask = 0xFF;
};

// species from its stored form F * species (F = 8 or 6, species < 8)
__device__ __forceinline__ int species_of(int v, int F) { return F == 8 ? v >> 3 : (v * 43) >> 8; }

// Padded copies of a replica: rows of conventional cells with a 2-cell
// periodic halo on every axis.  Interleaved rows hold the m basis sites of a
// cell side by side (byte m * (x + H) + b); basis-planar rows hold one column
// per basis site (byte b * cp + x + H), so that neighbouring link cells' sites
// of one basis are 4 bytes apart and a wave's LDS reads of them fall into
// distinct banks.
template <bool PLANAR>
__device__ __forceinline__ int row_byte(const RepDev& rep, int m, int x, int b)
{
    return PLANAR ? b * rep.cp + x + kHalo : m * (x + kHalo) + b;
}

// Write one species value to a site and to every periodic image of it that
// lies inside the padded copy.
template <bool PLANAR>
__device__ __forceinline__ void store_site(uint8_t* pad, const RepDev& rep, int m, int x, int y, int z,
                                           int b, uint8_t v)
{
    const int prow = PLANAR ? rep.prowp : rep.prow;
    if (x >= kHalo && x < rep.L[0] - kHalo && y >= kHalo && y < rep.L[1] - kHalo && z >= kHalo &&
        z < rep.L[2] - kHalo) {
        // away from the faces a site has no other image
        pad[((int64_t)(z + kHalo) * rep.prows + (y + kHalo)) * prow + row_byte<PLANAR>(rep, m, x, b)] = v;
        return;
    }
    int xs[3], ys[3], zs[3];
    int nx = 0, ny = 0, nz = 0;
    xs[nx++] = x;
    if (x < kHalo) xs[nx++] = x + rep.L[0];
    if (x >= rep.L[0] - kHalo) xs[nx++] = x - rep.L[0];
    ys[ny++] = y;
    if (y < kHalo) ys[ny++] = y + rep.L[1];
    if (y >= rep.L[1] - kHalo) ys[ny++] = y - rep.L[1];
    zs[nz++] = z;
    if (z < kHalo) zs[nz++] = z + rep.L[2];
    if (z >= rep.L[2] - kHalo) zs[nz++] = z - rep.L[2];
    for (int iz = 0; iz < nz; ++iz)
        for (int iy = 0; iy < ny; ++iy) {
            uint8_t* row = pad + ((int64_t)(zs[iz] + kHalo) * rep.prows + (ys[iy] + kHalo)) * prow;
            for (int ix = 0; ix < nx; ++ix) row[row_byte<PLANAR>(rep, m, xs[ix], b)] = v;
        }
}

// acc + (1 << sh) in one instruction (v_lshl_add): the packed counter gains
// one in the 8-bit field of the neighbour's species (sh = 8 * species).
__device__ __forceinline__ uint32_t shl1_add(uint32_t sh, uint32_t acc)
{
    uint32_t r;
    asm("v_lshl_add_u32 %0, 1, %1, %2" : "=v"(r) : "v"(sh), "v"(acc));
    return r;
}

__device__ __forceinline__ uint64_t shl1_add(uint32_t sh, uint64_t acc) { return acc + ((uint64_t)1 << sh); }

// Four of them in one asm block: the compiler pads every inline asm that
// writes a VGPR with a wait state, so a block per neighbour cost one per add.
__device__ __forceinline__ uint32_t shl1_add4(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t acc)
{
    uint32_t r;
    asm("v_lshl_add_u32 %0, 1, %1, %5\n\t"
        "v_lshl_add_u32 %0, 1, %2, %0\n\t"
        "v_lshl_add_u32 %0, 1, %3, %0\n\t"
        "v_lshl_add_u32 %0, 1, %4, %0"
        : "=&v"(r)
        : "v"(a), "v"(b), "v"(c), "v"(d), "v"(acc));
    return r;
}
__device__ __forceinline__ uint64_t shl1_add4(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint64_t acc)
{
    return shl1_add(d, shl1_add(c, shl1_add(b, shl1_add(a, acc))));
}
__device__ __forceinline__ uint32_t shl1_add2(uint32_t a, uint32_t b, uint32_t acc)
{
    uint32_t r;
    asm("v_lshl_add_u32 %0, 1, %1, %3\n\t"
        "v_lshl_add_u32 %0, 1, %2, %0"
        : "=&v"(r)
        : "v"(a), "v"(b), "v"(acc));
    return r;
}
__device__ __forceinline__ uint64_t shl1_add2(uint32_t a, uint32_t b, uint64_t acc) { return shl1_add(b, shl1_add(a, acc)); }

// Packed neighbour counters of a basis-B site at LDS byte `base`: A[s] gets
// 1 << (8 * species) per neighbour of shell s.  Offsets are compile-time
// displacements times the launch-uniform window pitches.
// The reads are rebased at the most negative offset (a window's neighbours lie
// within two conventional cells on every axis), so that every per-neighbour
// offset is a non-negative constant that fits the LDS instruction's immediate.
// Smallest cell offset on each axis and smallest basis index over the
// neighbours (all shells) of a basis-b site.
constexpr Nb min_components(const Geometry& G, int b)
{
    Nb r{0, 0, 0, b};
    for (int s = 0; s < kMaxShells; ++s)
        for (int n = 0; n < G.Z[s]; ++n) {
            const Nb nb = nb_of(G, b, G.v[s][n][0], G.v[s][n][1], G.v[s][n][2]);
            r.dx = nb.dx < r.dx ? nb.dx : r.dx;
            r.dy = nb.dy < r.dy ? nb.dy : r.dy;
            r.dz = nb.dz < r.dz ? nb.dz : r.dz;
            r.bt = nb.bt < r.bt ? nb.bt : r.bt;
        }
    return r;
}

template <int LAT, int B, bool PLANAR, typename CT>
__device__ __forceinline__ void count_uniform(const uint8_t* win, int base, int LP, int PL, int CP, int S,
                                              CT (&A)[kMaxShells])
{
    constexpr Geometry G = kGeom[LAT];
    // interleaved rows: x step m, basis step 1; basis-planar rows: x step 1, basis step CP
    const int XS = PLANAR ? 1 : G.m, BS = PLANAR ? CP : 1;
    // rebase at the smallest neighbour component on every axis (and basis):
    // the window holds every neighbour, so base + lo stays inside it
    constexpr Nb mn = min_components(G, B);
    const int lo = mn.dz * PL + mn.dy * LP + XS * mn.dx + BS * (mn.bt - B);
    // opaque to the compiler, so it keeps this base and every read's offset
    // (non-negative, below 64 KiB) goes into the instruction's offset field
    // instead of a per-read address add
    int rb = base + lo;
    asm("" : "+v"(rb));
    const uint8_t* w = win + rb;
    // all reads of a shell are issued before its counter chain starts, so
    // their LDS latencies overlap
#pragma unroll
    for (int s = 0; s < kMaxShells; ++s) {
        CT acc = 0;
        if (s < S) {
            uint32_t v[kMaxZ];
#pragma unroll
            for (int n = 0; n < G.Z[s]; ++n) {
                const Nb nb = nb_of(G, B, G.v[s][n][0], G.v[s][n][1], G.v[s][n][2]);
                const int off = nb.dz * PL + nb.dy * LP + XS * nb.dx + BS * (nb.bt - B);
                v[n] = w[off - lo];
            }
            const int Z4 = G.Z[s] & ~3;
#pragma unroll
            for (int n = 0; n < Z4; n += 4) acc = shl1_add4(v[n], v[n + 1], v[n + 2], v[n + 3], acc);
#pragma unroll
            for (int n = Z4; n < G.Z[s]; ++n) acc = shl1_add(v[n], acc);
        }
        A[s] = acc;
    }
}

// Both sites of a BCC trial (active site of basis B at `ba`, its partner of
// the other basis at `bb`): the same counts as two count_uniform calls, with
// the window reads software-pipelined in chunks of up to CHUNK neighbours of
// one (site, shell): the reads of chunk g + 1 are issued before chunk g's
// counter adds (scheduling barriers keep that order), so LDS latency
// overlaps the adds.  Row windows (compile-time pitches in the benchmark's
// preset) take chunks of 4: 954 us per 800^3 launch against 984 for whole
// (site, shell) groups, 965 for chunks of 8, 960 for chunks of 4 with two in
// flight, 972 with the order left to the compiler.  Tile windows keep whole
// groups: with chunks of 4 their runtime-pitch address arithmetic is cut
// into the same small pieces, and the batched tile sweeps of the ladder ran
// 11 % slower.
struct PairChunk {
    int site, shell, n0, n1;  // neighbours n0 .. n1 - 1 of shell `shell` of site 0 (active) or 1 (partner)
};
struct PairChunks {
    int n;
    PairChunk c[2 * kMaxShells * kMaxZ];
};
constexpr PairChunks make_pair_chunks(const Geometry& G, int S, int chunk)
{
    PairChunks P{};
    P.n = 0;
    for (int site = 0; site < 2; ++site)
        for (int s = 0; s < S; ++s)
            for (int n0 = 0; n0 < G.Z[s]; n0 += chunk) {
                PairChunk c{};
                c.site = site;
                c.shell = s;
                c.n0 = n0;
                c.n1 = n0 + chunk < G.Z[s] ? n0 + chunk : G.Z[s];
                P.c[P.n++] = c;
            }
    return P;
}

template <int LAT, int B, bool PLANAR, typename CT, int CHUNK>
__device__ __forceinline__ void count_pair(const uint8_t* win, int ba, int bb, int LP, int PL, int CP, int S,
                                           CT (&A)[kMaxShells], CT (&Bc)[kMaxShells])
{
    constexpr Geometry G = kGeom[LAT];
    constexpr int BB = 1 - B;
    const int XS = PLANAR ? 1 : G.m, BS = PLANAR ? CP : 1;
    constexpr Nb mna = min_components(G, B), mnb = min_components(G, BB);
    const int loa = mna.dz * PL + mna.dy * LP + XS * mna.dx + BS * (mna.bt - B);
    const int lob = mnb.dz * PL + mnb.dy * LP + XS * mnb.dx + BS * (mnb.bt - BB);
    int ra = ba + loa, rb = bb + lob;
    asm("" : "+v"(ra), "+v"(rb));
    const uint8_t* wa = win + ra;
    const uint8_t* wb = win + rb;
    // every chunk of the largest shell count; chunks of shells >= S are skipped
    constexpr PairChunks PC = make_pair_chunks(G, kMaxShells, CHUNK);
#pragma unroll
    for (int s = 0; s < kMaxShells; ++s) {
        A[s] = 0;
        Bc[s] = 0;
    }
    uint32_t buf[2][CHUNK];
    auto load = [&](const int g, uint32_t(&v)[CHUNK]) {
        const PairChunk& c = PC.c[g];
        const int bs = c.site == 0 ? B : BB;
        if (c.shell < S) {
#pragma unroll
            for (int n = c.n0; n < c.n1; ++n) {
                const Nb nb = nb_of(G, bs, G.v[c.shell][n][0], G.v[c.shell][n][1], G.v[c.shell][n][2]);
                const int off = nb.dz * PL + nb.dy * LP + XS * nb.dx + BS * (nb.bt - bs);
                v[n - c.n0] = c.site == 0 ? wa[off - loa] : wb[off - lob];
            }
        }
    };
    auto add = [&](const int g, const uint32_t(&v)[CHUNK]) {
        const PairChunk& c = PC.c[g];
        if (c.shell < S) {
            CT acc = c.site == 0 ? A[c.shell] : Bc[c.shell];
            const int Z = c.n1 - c.n0, Z4 = Z & ~3;
#pragma unroll
            for (int n = 0; n < Z4; n += 4) acc = shl1_add4(v[n], v[n + 1], v[n + 2], v[n + 3], acc);
            if (Z - Z4 >= 2) {
                acc = shl1_add2(v[Z4], v[Z4 + 1], acc);
                if (Z - Z4 == 3) acc = shl1_add(v[Z4 + 2], acc);
            } else if (Z - Z4 == 1) {
                acc = shl1_add(v[Z4], acc);
            }
            if (c.site == 0) A[c.shell] = acc;
            else Bc[c.shell] = acc;
        }
    };
    load(0, buf[0]);
#pragma unroll
    for (int g = 0; g < PC.n; ++g) {
        if (g + 1 < PC.n) load(g + 1, buf[(g + 1) & 1]);
        __builtin_amdgcn_sched_barrier(0);
        add(g, buf[g & 1]);
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Same for the partner of an FCC site: per-lane offsets (relative to the
// active site) from an LDS table, since the partner basis varies per lane.
template <int LAT, typename CT>
__device__ __forceinline__ void count_table(const uint8_t* win, int base, const int16_t* offs, int S,
                                            CT (&A)[kMaxShells])
{
    constexpr Geometry G = kGeom[LAT];
    int j = 0;
#pragma unroll
    for (int s = 0; s < kMaxShells; ++s) {
        CT acc = 0;
        if (s < S) {
#pragma unroll
            for (int n = 0; n < G.Z[s]; ++n) acc = shl1_add(win[base + offs[j + n]], acc);
        }
        j += G.Z[s];
        A[s] = acc;
    }
}

struct Lds {
    const double* D;
    const int32_t* Q;  // integer dE terms [S][K][K][K], then bias sums [K][K]
    float qscale;      // value of one integer unit (a power of two)
    float qeps;        // bound on |integer dE - binary64 dE| before the float conversion
    const int16_t* offP;
    const int32_t* offB;
    const int8_t* pd;
};

__device__ __forceinline__ Lds lds_ptrs(const SweepArgs& A, uint8_t* smem)
{
    Lds l;
    l.D = (const double*)(smem + A.lds_d);
    l.Q = (const int32_t*)(smem + A.lds_q);
    // read at run time, like the tables, so that a captured graph follows smcx_set_epi
    using CI = const __attribute__((address_space(4))) int32_t;
    const int nq = A.S * A.K * A.K * A.K + A.K * A.K;
    l.qscale = __int_as_float(((CI*)A.Qtab)[nq]);
    l.qeps = __int_as_float(((CI*)A.Qtab)[nq + 1]);
    l.offP = (const int16_t*)(smem + A.lds_offp);
    l.offB = (const int32_t*)(smem + A.lds_offb);
    l.pd = (const int8_t*)(smem + A.lds_pd);
    return l;
}

// Copy the launch tables into LDS (a barrier follows before first use).
template <int LAT>
__device__ void load_tables(const SweepArgs& A, uint8_t* smem)
{
    constexpr int m = kGeom[LAT].m;
    double* D = (double*)(smem + A.lds_d);
    const int nD = A.K * A.K * A.S * A.K;
    for (int i = threadIdx.x; i < nD; i += blockDim.x) D[i] = A.Dtab[i];
    int32_t* Q = (int32_t*)(smem + A.lds_q);
    const int nQ = nD + A.K * A.K;
    for (int i = threadIdx.x; i < nQ; i += blockDim.x) Q[i] = A.Qtab[i];
    if constexpr (LAT == SMCX_FCC) {
        int16_t* P = (int16_t*)(smem + A.lds_offp);
        const int nP = m * A.Z1 * A.sumZ;
        for (int i = threadIdx.x; i < nP; i += blockDim.x) P[i] = A.offP[i];
    }
    int32_t* Bo = (int32_t*)(smem + A.lds_offb);
    int8_t* pd = (int8_t*)(smem + A.lds_pd);
    for (int i = threadIdx.x; i < m * A.Z1; i += blockDim.x) Bo[i] = A.offB[i];
    for (int i = threadIdx.x; i < 4 * m * A.Z1; i += blockDim.x) pd[i] = A.pdisp[i];
}

// ---------------------------------------------------------------------------
// Window geometry policies.  GeoRt reads tile shape and window pitches from
// the launch arguments (any partition); GeoFix<...> fixes them at compile
// time for uniform partitions, so that every LDS neighbour offset is an
// immediate and cell origins are c * ELL.
// ---------------------------------------------------------------------------
struct GeoRt {
    static constexpr bool fixed = false;
    static constexpr bool rows = false;
    static constexpr bool own_cp = false;
    static constexpr bool may_alias = true;  // a partner may have images in other shells (an edge of 2)
    static constexpr int ELL = 0;
    __device__ static int T(const SweepArgs& A, int a) { return A.T[a]; }
    __device__ static int LP(const SweepArgs& A) { return A.LP; }
    __device__ static int WY(const SweepArgs& A) { return A.WY; }
    __device__ static int WZ(const SweepArgs& A) { return A.WZ; }
    __device__ static int block(const SweepArgs&) { return blockDim.x; }
    __device__ static int K(const SweepArgs& A) { return A.K; }
    __device__ static int S(const SweepArgs& A) { return A.S; }
    __device__ static int CP(const RepDev& rep) { return rep.cp; }
};

template <int PI>
struct GeoFix {
    static constexpr Preset P = kPresets[PI];
    static_assert(preset_ok(P), "tile start must be 16-byte aligned");
    static constexpr bool fixed = true;
    static constexpr bool rows = false;
    static constexpr bool own_cp = false;
    static constexpr bool may_alias = true;
    static constexpr int ELL = P.ell;
    static constexpr int kLP = preset_LP(P), kWY = preset_WY(P), kWZ = preset_WZ(P);
    static constexpr int kBLOCK = (P.tx * P.ty * P.tz + 63) / 64 * 64;
    __device__ static constexpr int T(const SweepArgs&, int a) { return a == 0 ? P.tx : (a == 1 ? P.ty : P.tz); }
    __device__ static constexpr int LP(const SweepArgs&) { return preset_LP(P); }
    __device__ static constexpr int WY(const SweepArgs&) { return preset_WY(P); }
    __device__ static constexpr int WZ(const SweepArgs&) { return preset_WZ(P); }
    __device__ static constexpr int block(const SweepArgs&) { return (P.tx * P.ty * P.tz + 63) / 64 * 64; }
    __device__ static constexpr int K(const SweepArgs&) { return P.K; }
    __device__ static constexpr int S(const SweepArgs&) { return P.S; }
    __device__ static int CP(const RepDev& rep) { return rep.cp; }  // tile windows are interleaved
};

// Row windows: the window holds whole padded x-rows (periodic images of the
// sites within two cells of the x faces included), so a written site must be
// copied to its image in the window too.  KK / SS fix the species and shell
// counts at compile time (0: taken from the launch).
template <int KK, int SS>
struct GeoRow : GeoRt {
    static constexpr bool rows = true;
    static constexpr bool own_cp = true;  // replicas may differ in column pitch
    __device__ static int K(const SweepArgs& A) { return KK ? KK : A.K; }
    __device__ static int S(const SweepArgs& A) { return SS ? SS : A.S; }
};

// Row windows of a compile-time preset.
template <int PI>
struct GeoRowFix : GeoRt {
    static constexpr RowPreset P = kRowPresets[PI];
    static constexpr bool rows = true;
    static constexpr bool may_alias = false;  // chosen only for lattices without partner images
    __device__ static constexpr int T(const SweepArgs&, int a) { return a == 0 ? P.rt0 : (a == 1 ? P.rt1 : P.rt2); }
    __device__ static constexpr int LP(const SweepArgs&) { return P.LP; }
    __device__ static constexpr int WY(const SweepArgs&) { return P.WY; }
    __device__ static constexpr int WZ(const SweepArgs&) { return P.WZ; }
    __device__ static constexpr int K(const SweepArgs&) { return P.K; }
    __device__ static constexpr int S(const SweepArgs&) { return P.S; }
    __device__ static constexpr int CP(const RepDev&) { return P.cp; }
};

struct TileGeom {
    int w0[3];   // window origin (replica conventional cells, >= -H)
    int n[3];    // window extent
    int gx0;     // first staged byte of each padded row
    int c0[3];   // first link cell of the tile
    int c1[3];   // one past the last link cell
};

template <class Geo>
__device__ __forceinline__ int cell_origin(const SweepArgs& A, const RepDev& rep, int a, int c)
{
    if constexpr (Geo::fixed) {
        return c * Geo::ELL;
    } else {
        const int32_t* org = A.origins + rep.cs_off;
        if (a > 0) org += rep.nc[0] + 1;
        if (a > 1) org += rep.nc[1] + 1;
        return org[c];
    }
}

// Window of one tile for mini-step offsets o, identical in every thread.
// Returns false when no cell of the tile has these offsets.
template <int LAT, class Geo>
__device__ __forceinline__ bool tile_geometry(const SweepArgs& A, const RepDev& rep, int64_t tile,
                                              const int (&o)[3], TileGeom& tg)
{
    constexpr int m = kGeom[LAT].m;
    // tiles per replica stay below 2^31 (cells per replica do), so 32-bit division
    const int tl = (int)tile;
    const int tx = tl % rep.ntile[0];
    const int trest = tl / rep.ntile[0];
    const int ty = trest % rep.ntile[1];
    const int tz = trest / rep.ntile[1];
    tg.c0[0] = tx * Geo::T(A, 0);
    tg.c0[1] = ty * Geo::T(A, 1);
    tg.c0[2] = tz * Geo::T(A, 2);
    bool any = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        tg.c1[a] = min(tg.c0[a] + Geo::T(A, a), rep.nc[a]);
        tg.w0[a] = cell_origin<Geo>(A, rep, a, tg.c0[a]) + o[a] - kHalo;
        const int w1 = min(cell_origin<Geo>(A, rep, a, tg.c1[a] - 1) + o[a] + kHalo + 1, rep.L[a] + kHalo);
        tg.n[a] = w1 - tg.w0[a];
        any &= tg.n[a] > 0;
        if constexpr (!Geo::fixed) {
            // some cell of the tile must be longer than the offset (uneven partitions)
            bool has = false;
            for (int c = tg.c0[a]; c < tg.c1[a]; ++c)
                has |= cell_origin<Geo>(A, rep, a, c + 1) - cell_origin<Geo>(A, rep, a, c) > o[a];
            any &= has;
        }
    }
    tg.gx0 = (m * (tg.w0[0] + kHalo)) & ~15;
    return any;
}

// Issue the window loads of a tile straight into LDS (global_load_lds_dwordx4:
// lane i of a wave writes the 16 bytes at M0 + 16 i).  Window row R (plane
// R / WY, row R % WY) occupies LP bytes at buf + R LP.  Long rows go a wave
// per row (R = wave, wave + waves, ...): the row's source address is
// wave-uniform and a lane's part of it 16 bytes per chunk.  Short rows would
// leave most lanes of such a wave idle, so there window slot j (16 bytes at
// buf + 16 j: row j / (LP / 16), chunk j % (LP / 16)) goes to thread j, j +
// block, ..., each advancing its source address by fixed steps.  Blocks are
// whole waves.  The loads complete asynchronously; the caller waits on vmcnt
// and a barrier before reading the buffer.
template <int LAT, class Geo>
__device__ __forceinline__ void stage_async(const SweepArgs& A, const RepDev& rep, const TileGeom& tg,
                                            const uint8_t* pad, uint8_t* buf)
{
    constexpr int m = kGeom[LAT].m;
    const int LP = Geo::LP(A), LPc = LP >> 4;
    const int WY = Geo::WY(A);
    const int nrows = Geo::WZ(A) * WY;
    // row windows hold whole basis-planar rows; tile windows a byte range of
    // interleaved rows
    const int grow = Geo::rows ? rep.prowp : rep.prow;
    const int gx1 = Geo::rows ? rep.prowp : (m * (tg.w0[0] + tg.n[0] + kHalo) + 15) & ~15;
    const int n16 = min((gx1 - tg.gx0) >> 4, LPc);  // chunks of a row, never past the window's pitch
    // the window geometry is the same in every lane: scalar registers keep
    // the loops and the row addresses out of vector code
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int block = __builtin_amdgcn_readfirstlane(Geo::block(A));
    const int n1 = __builtin_amdgcn_readfirstlane(tg.n[1]), n2 = __builtin_amdgcn_readfirstlane(tg.n[2]);
    const uint64_t off = (uint64_t)(((int64_t)(tg.w0[2] + kHalo) * rep.prows + (tg.w0[1] + kHalo)) * grow + tg.gx0);
    const uint8_t* base = pad + (int64_t)(((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(off >> 32)) << 32) |
                                          __builtin_amdgcn_readfirstlane((uint32_t)off));
    const int64_t plane = (int64_t)rep.prows * grow;
    if (n16 >= 40) {
        const int nwaves = block >> 6;
        int wz = wave / WY, wy = wave - wz * WY;
        for (int R = wave; R < nrows; R += nwaves) {
            if (wy < n1 && wz < n2) {
                const uint8_t* row = base + wz * plane + (int64_t)wy * grow;
                for (int cb = 0; cb < n16; cb += 64)
                    if (cb + lane < n16)
                        __builtin_amdgcn_global_load_lds(
                            (const __attribute__((address_space(1))) void*)(row + 16 * (cb + lane)),
                            (__attribute__((address_space(3))) void*)(buf + R * LP + 16 * cb), 16, 0, 0);
            }
            wy += nwaves;
            while (wy >= WY) {
                wy -= WY;
                ++wz;
            }
        }
        return;
    }
    const int nslots = nrows * LPc;
    int j = wave * 64 + lane;
    int R = j / LPc, col = j - R * LPc;
    int wz = R / WY, wy = R - wz * WY;
    const int dR = block / LPc, dcol = block - dR * LPc;
    const uint8_t* src = base + wz * plane + (int64_t)wy * grow + 16 * col;
    const int64_t step = (int64_t)dR * grow + 16 * dcol, wrap_col = grow - 16 * LPc, wrap_row = plane - (int64_t)WY * grow;
    for (int jb = wave * 64; jb < nslots; jb += block) {
        if (jb + lane < nslots && col < n16 && wy < n1 && wz < n2)
            __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                             (__attribute__((address_space(3))) void*)(buf + 16 * jb), 16, 0, 0);
        col += dcol;
        wy += dR;
        src += step;
        if (col >= LPc) {
            col -= LPc;
            ++wy;
            src += wrap_col;
        }
        while (wy >= WY) {
            wy -= WY;
            ++wz;
            src += wrap_row;
        }
    }
}

// Per-thread staging plan of a compile-time window: thread t stages window
// slots t + i * BLOCK; soff[i] is the slot's byte offset from the window's
// first staged byte in the padded copy (plane and row pitches of a replica).
template <int LAT, class Geo>
struct StagePlan {
    static constexpr int LPc = Geo::kLP / 16;
    static constexpr int WY = Geo::kWY;
    static constexpr int WZ = Geo::kWZ;
    static constexpr int NSLOT = WZ * WY * LPc;
    static constexpr int BLOCK = Geo::kBLOCK;
    static constexpr int NP = (NSLOT + BLOCK - 1) / BLOCK;
    int soff[NP];
    int rep = -1;

    __device__ __forceinline__ void prepare(const RepDev& rp, int r)
    {
        if (r == rep) return;
        rep = r;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int slot = threadIdx.x + i * BLOCK;
            const int R = slot / LPc, col = slot - R * LPc;
            const int wz = R / WY, wy = R - wz * WY;
            soff[i] = (wz * rp.prows + wy) * rp.prow + 16 * col;
        }
    }

    // every slot of a full window lies inside the padded copy
    __device__ __forceinline__ void stage_full(const uint8_t* first, uint8_t* buf) const
    {
        const int wave64 = __builtin_amdgcn_readfirstlane(threadIdx.x & ~63);
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            if (i * BLOCK + wave64 < NSLOT && threadIdx.x + i * BLOCK < NSLOT)
                __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(first + soff[i]),
                                                 (__attribute__((address_space(3))) void*)(buf + 16 * (i * BLOCK + wave64)),
                                                 16, 0, 0);
        }
    }
};

// A trial is split at the point where it stops reading the tile window:
// trial_read draws the random numbers and forms the packed neighbour counts
// from LDS, trial_finish turns them into dE, takes the Metropolis decision
// and writes the swap.  Between the two the window buffer may be refilled.
template <int E>
struct LaneState {
    using CT = typename Enc<E>::T;
    int active = 0;
    int p8 = 0, q8 = 0, k = 0, b = 0;
    CT Ca[kMaxShells], Cb[kMaxShells];
    uint32_t w1 = 0, w2 = 0;
    int ax = 0, ay = 0, az = 0;
    int la = 0, lb = 0;  // window bytes of the two sites
    int64_t ia = 0;
};

template <int LAT, int E, int B, class Geo>
__device__ __forceinline__ void trial_read(const SweepArgs& A, const RepDev& rep, const Lds& T, const uint8_t* win,
                                           const TileGeom& tg, int r, uint32_t t, int ax, int ay, int az,
                                           LaneState<E>& L, int64_t yz = 0)
{
    using CT = typename Enc<E>::T;
    constexpr Geometry G = kGeom[LAT];
    constexpr int m = G.m;
    constexpr int Z1 = G.Z[0];
    const int LP = Geo::LP(A), WY = Geo::WY(A), PL = LP * WY;
    const int S = Geo::S(A);
    constexpr bool PLANAR = Geo::rows;
    const int la = ((az - tg.w0[2]) * WY + (ay - tg.w0[1])) * LP +
                   (PLANAR ? B * Geo::CP(rep) + ax + kHalo : m * (ax + kHalo) + B) - tg.gx0;
    // site index b + m (x + L0 (y + L1 z)); row kernels pass yz = m L0 (y + L1 z),
    // fixed for a row group, so a trial adds only b + m x
    int64_t ia;
    if constexpr (Geo::rows)
        ia = yz + (B + m * ax);
    else
        ia = B + (int64_t)m * (ax + (int64_t)rep.L[0] * (ay + (int64_t)rep.L[1] * az));
    uint32_t w0, w1, w2, w3;
    philox4x32_10((uint32_t)ia, (uint32_t)((uint64_t)ia >> 32), t, (uint32_t)r, (uint32_t)A.seed,
                  (uint32_t)(A.seed >> 32), w0, w1, w2, w3);
    (void)w3;
    const int k = (int)__umulhi(w0, (uint32_t)Z1);
    const int p8 = win[la];
    int offb;
    if constexpr (Geo::own_cp && LAT == SMCX_BCC) {
        // the partner's window offset from its cell displacement and this
        // replica's column pitch (row windows of replicas of different widths)
        const int8_t* q = T.pd + (B * Z1 + k) * 4;
        offb = q[2] * PL + q[1] * LP + q[0] + (q[3] - B) * Geo::CP(rep);
    } else {
        offb = T.offB[B * Z1 + k];
    }
    const int q8 = win[la + offb];
    L.active = 1;
    L.p8 = p8;
    L.q8 = q8;
    L.k = k;
    L.b = B;
    L.w1 = w1;
    L.w2 = w2;
    L.ax = ax;
    L.ay = ay;
    L.az = az;
    L.ia = ia;
    L.la = la;
    L.lb = la + offb;
    if (p8 == q8) return;
    if constexpr (LAT == SMCX_BCC) {
        // the partner of a BCC site always sits on the other sublattice
        count_pair<LAT, B, PLANAR, CT, Geo::rows ? 4 : kMaxZ>(win, la, la + offb, LP, PL, Geo::CP(rep), S, L.Ca, L.Cb);
    } else {
        count_uniform<LAT, B, PLANAR, CT>(win, la, LP, PL, Geo::CP(rep), S, L.Ca);
        count_table<LAT, CT>(win, la, T.offP + (B * Z1 + k) * A.sumZ, S, L.Cb);
    }
}

// The decision of a trial the integer screen leaves open (a few in 1e5 at
// the benchmark's temperature): dE summed in binary64, s and t ascending, from
// D[s][t][p][q] (Dp points at the lane's (p, q) entry), then the float screen
// and, where that cannot decide either, exp in binary64, the test u < P and
// the near-tie check.  The sum starts from the first product rather than from
// +0.0 + it: the two differ only in the sign of a zero sum, and dE <= 0
// accepts either.  Out of line: inlined, its registers would weigh on every
// trial's code.  Returns bit 0: accepted, bit 1: near-tie.
template <int E>
__device__ __noinline__ int decide_binary64(const double* Dp, typename Enc<E>::T d0, typename Enc<E>::T d1,
                                            typename Enc<E>::T d2, typename Enc<E>::T d3, int K, int S, double beta,
                                            uint32_t w1, uint32_t w2)
{
    using EN = Enc<E>;
    using CT = typename EN::T;
    double dE = 0.0;
    bool first = true;
    for (int s = 0; s < S; ++s) {
        CT f = s == 0 ? d0 : (s == 1 ? d1 : (s == 2 ? d2 : d3));
        const double* Ds = Dp + s * K * K * K;
        for (int tt = 0; tt < K; ++tt) {
            const int c = (int)(f & EN::mask) - EN::half;
            const double term = (double)c * Ds[tt * K * K];
            dE = first ? term : dE + term;
            first = false;
            f >>= EN::F;
        }
    }
    if (dE <= 0.0) return 1;
    const double x = beta * dE;
    // A float estimate settles u < exp(-x) whenever u lies farther from it
    // than the estimate's error: the binary64 test then gives the same answer
    // and the trial is no near-tie.  For x <= 30, rounding x and x log2(e) to
    // float moves the exponent by < 8e-6, so exp2 is off by < 6e-6 relative
    // (plus an ulp or two of v_exp_f32); the margin is 1e-4 relative plus
    // 1e-9 for u's truncation and rounding.
    if (x > 30.0) {
        if (w1 != 0) return 0;
    } else {
        const float uf = (float)w1 * 0x1p-32f;
        const float Pf = __builtin_amdgcn_exp2f((float)x * -1.44269504f);
        if (fabsf(uf - Pf) > 1e-4f * Pf + 1e-9f) return uf < Pf ? 1 : 0;
    }
    const double P = exp(-x);
    const double u = (double)(((uint64_t)w1 << 21) | (uint64_t)(w2 >> 11)) * 0x1p-53;
    return (u < P ? 1 : 0) | (fabs(u - P) < 1e-12 ? 2 : 0);
}

// Returns flags: bit0 active, bit1 accepted, bit2 near-tie (0 for an idle lane).
template <int LAT, int E, class Geo>
__device__ __forceinline__ int trial_finish(const SweepArgs& A, const RepDev& rep, uint8_t* pad, const Lds& T,
                                            uint8_t* win, int r, uint32_t t, double beta, const LaneState<E>& L)
{
    using EN = Enc<E>;
    using CT = typename EN::T;
    constexpr Geometry G = kGeom[LAT];
    constexpr int m = G.m;
    constexpr int Z1 = G.Z[0];
    if (!L.active) return 0;
    if (L.p8 == L.q8) return 1;
    const int K = Geo::K(A), S = Geo::S(A);
    const int p8 = L.p8, q8 = L.q8, k = L.k;
    // species were checked < K at init; the clamp keeps table reads in bounds regardless
    const int p = min(species_of(p8, EN::F), K - 1), q = min(species_of(q8, EN::F), K - 1);
    // the per-shell count differences, fields biased by `half`
    CT dsh[kMaxShells];
#pragma unroll
    for (int s = 0; s < kMaxShells; ++s) {
        // images of the partner inside shell s (1, 0, 0, 0 unless an edge is 2)
        const CT mu = Geo::may_alias && rep.alias ? (CT)rep.mult[s][k] : (CT)(s == 0 ? 1 : 0);
        dsh[s] = s < S ? L.Ca[s] + EN::bias - L.Cb[s] + (mu << p8) - (mu << q8) : (CT)0;
    }
    // Screen: dE in integers.  Qtab holds every D[s][t][p][q] rounded to a
    // multiple of qscale (24-bit signed), so sum_t (c_t + half) Q - bias, bias
    // = half sum Q, is sum_t c_t Q exactly (modulo 2^32, and it fits in 32
    // bits), within qeps / qscale units of the binary64 dE.  It settles the
    // decision whenever that uncertainty cannot change it; otherwise the
    // binary64 sum and test below decide, as they always would.
    const int32_t* Qp = T.Q + (p * K + q);
    // every table read is issued before the first product, so the trial
    // waits for the LDS once
    int32_t qv[kMaxShells][EN::KP];
    const int32_t qbias = T.Q[S * K * K * K + p * K + q];
#pragma unroll
    for (int s = 0; s < kMaxShells; ++s)
#pragma unroll
        for (int tt = 0; tt < EN::KP; ++tt) qv[s][tt] = s < S && tt < K ? Qp[(s * K + tt) * K * K] : 0;
    __builtin_amdgcn_sched_barrier(0);
    uint32_t qacc = 0u - (uint32_t)qbias;
#pragma unroll
    for (int s = 0; s < kMaxShells; ++s) {
        if (s < S) {
#pragma unroll
            for (int tt = 0; tt < EN::KP; ++tt) {
                if (tt < K) {
                    const int u = (int)((dsh[s] >> (EN::F * tt)) & EN::mask);
                    qacc += (uint32_t)__mul24(u, qv[s][tt]);
                }
            }
        }
    }
    const float e = (float)(int32_t)qacc * T.qscale;
    const float eps = T.qeps + fabsf(e) * 0x1p-22f;
    const float bf = (float)beta;
    bool acc = false;
    bool tie = false;
    bool settled = true;
    if (e <= -eps) {
        acc = true;  // dE <= e + eps <= 0
    } else if (e > eps && bf >= 0.0f && bf * eps < 0.25f) {
        // dE > 0 and beta dE lies in [bf (e - eps), bf (e + eps)] up to float
        // rounding.  u = (w1 2^21 + (w2 >> 11)) 2^-53 lies in [w1 2^-32,
        // (w1 + 1) 2^-32).  With y = bf eps <= 1/4, exp(-beta dE) is within
        // a factor exp(+-y) (<= 1.14 y relative) of exp(-bf e), and the float
        // estimate of that is within 2e-5 relative for beta dE <= 31, so a
        // margin of 1e-4 + 1.2 y relative plus 1e-9 for u's truncation
        // settles u < exp(-beta dE) exactly, and such a trial is no near-tie.
        if (bf * (e - eps) * (1.0f - 0x1p-20f) > 30.0f) {
            // exp(-beta dE) < 1e-13, while u >= 2^-32 unless w1 == 0
            settled = L.w1 != 0;
        } else {
            const float uf = (float)L.w1 * 0x1p-32f;
            const float Pf = __builtin_amdgcn_exp2f(bf * e * -1.44269504f);
            settled = fabsf(uf - Pf) > (1e-4f + 1.2f * bf * eps) * Pf + 1e-9f;
            acc = uf < Pf;
        }
    } else {
        settled = false;
    }
    if (!settled) {
        static_assert(kMaxShells == 4, "four shell counters");
        const int f = decide_binary64<E>(T.D + (p * K + q), dsh[0], dsh[1], dsh[2], dsh[3], K, S, beta, L.w1, L.w2);
        acc = (f & 1) != 0;
        tie = (f & 2) != 0;
    }
    if (tie) {
        const int slot = atomicAdd(A.tie_count, 1);
        if (slot < A.tie_cap) {
            smcx_tie e;
            e.replica = r;
            e.sweep = t;
            e.site = L.ia;
            e.decision = acc ? 1 : 0;
            e.pad = 0;
            A.ties[slot] = e;
        }
    }
    if (acc) {
        const int8_t* pd = T.pd + (L.b * Z1 + k) * 4;
        int bx = L.ax + pd[0], by = L.ay + pd[1], bz = L.az + pd[2];
        const int bb = pd[3];
        const int ubx = bx;  // partner x before the periodic wrap (its column in a row window)
        bx += bx < 0 ? rep.L[0] : (bx >= rep.L[0] ? -rep.L[0] : 0);
        by += by < 0 ? rep.L[1] : (by >= rep.L[1] ? -rep.L[1] : 0);
        bz += bz < 0 ? rep.L[2] : (bz >= rep.L[2] ? -rep.L[2] : 0);
        // the padded copy holds F * species, like the window; the window copy
        // serves the next basis site's trial of this lane
        // (row windows reach HBM in one copy of their changed rows per group)
        if constexpr (!Geo::rows) {
            store_site<false>(pad, rep, m, L.ax, L.ay, L.az, L.b, (uint8_t)q8);
            store_site<false>(pad, rep, m, bx, by, bz, bb, (uint8_t)p8);
        }
        win[L.la] = (uint8_t)q8;
        win[L.lb] = (uint8_t)p8;
        if constexpr (Geo::rows) {
            // row windows span x in [-H, L + H): sites within H of an x face appear twice
            const int Lx = rep.L[0], sh = Lx;  // basis-planar rows: x step 1
            if (L.ax < kHalo) win[L.la + sh] = (uint8_t)q8;
            if (L.ax >= Lx - kHalo) win[L.la - sh] = (uint8_t)q8;
            if (ubx < kHalo) win[L.lb + sh] = (uint8_t)p8;
            if (ubx >= Lx - kHalo) win[L.lb - sh] = (uint8_t)p8;
        }
    }
    return 1 | (acc ? 2 : 0) | (tie ? 4 : 0);
}

template <int LAT, int E, class Geo>
__device__ __forceinline__ void read_dispatch(int b, const SweepArgs& A, const RepDev& rep, const Lds& T,
                                              const uint8_t* win, const TileGeom& tg, int r, uint32_t t, int ax,
                                              int ay, int az, LaneState<E>& L)
{
    if constexpr (LAT == SMCX_BCC) {
        if (b == 0) trial_read<LAT, E, 0, Geo>(A, rep, T, win, tg, r, t, ax, ay, az, L);
        else trial_read<LAT, E, 1, Geo>(A, rep, T, win, tg, r, t, ax, ay, az, L);
    } else {
        switch (b) {
        case 0: trial_read<LAT, E, 0, Geo>(A, rep, T, win, tg, r, t, ax, ay, az, L); break;
        case 1: trial_read<LAT, E, 1, Geo>(A, rep, T, win, tg, r, t, ax, ay, az, L); break;
        case 2: trial_read<LAT, E, 2, Geo>(A, rep, T, win, tg, r, t, ax, ay, az, L); break;
        default: trial_read<LAT, E, 3, Geo>(A, rep, T, win, tg, r, t, ax, ay, az, L); break;
        }
    }
}

// Per-thread trial statistics, flushed with one wave reduction and three
// atomics per wave.
struct Stats {
    int att = 0, acc = 0, tie = 0;
};

__device__ __forceinline__ int wave_sum_i(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ void flush_stats(const SweepArgs& A, int r, Stats& st)
{
    const int a = wave_sum_i(st.att), c = wave_sum_i(st.acc), t = wave_sum_i(st.tie);
    if ((threadIdx.x & 63) == 0 && r >= 0) {
        unsigned long long* p = (unsigned long long*)(A.stats + 3 * (int64_t)r);
        if (a) atomicAdd(p + 0, (unsigned long long)a);
        if (c) atomicAdd(p + 1, (unsigned long long)c);
        if (t) atomicAdd(p + 2, (unsigned long long)t);
    }
    st = Stats();
}

// The same for a whole workgroup at a point every thread reaches: the waves'
// sums meet in LDS and one thread adds them to the replica's counters (one
// global atomic per counter and workgroup instead of per wave).
__device__ __forceinline__ void flush_stats_block(const SweepArgs& A, int r, Stats& st)
{
    __shared__ int red[3];
    if (threadIdx.x == 0) red[0] = red[1] = red[2] = 0;
    __syncthreads();
    const int a = wave_sum_i(st.att), c = wave_sum_i(st.acc), t = wave_sum_i(st.tie);
    if ((threadIdx.x & 63) == 0) {
        if (a) atomicAdd(&red[0], a);
        if (c) atomicAdd(&red[1], c);
        if (t) atomicAdd(&red[2], t);
    }
    __syncthreads();
    if (threadIdx.x == 0 && r >= 0) {
        unsigned long long* p = (unsigned long long*)(A.stats + 3 * (int64_t)r);
        if (red[0]) atomicAdd(p + 0, (unsigned long long)red[0]);
        if (red[1]) atomicAdd(p + 1, (unsigned long long)red[1]);
        if (red[2]) atomicAdd(p + 2, (unsigned long long)red[2]);
    }
    st = Stats();
}

// Block barrier that orders LDS accesses only: global loads issued before it
// stay in flight (a full __syncthreads also drains them).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// First half of the trials of one staged tile (one lane per link cell):
// lanes outside the tile or whose cell is shorter than an offset stay idle.
template <int LAT, int E, class Geo>
__device__ __forceinline__ void tile_read(const SweepArgs& A, const RepDev& rep, int r, const TileGeom& tg, int b,
                                          const int (&o)[3], uint32_t t, const Lds& T, const uint8_t* win,
                                          LaneState<E>& L)
{
    L.active = 0;
    const int l = threadIdx.x;
    const int lx = l % Geo::T(A, 0);
    const int ly = (l / Geo::T(A, 0)) % Geo::T(A, 1);
    const int lz = l / (Geo::T(A, 0) * Geo::T(A, 1));
    const int cx = tg.c0[0] + lx, cy = tg.c0[1] + ly, cz = tg.c0[2] + lz;
    if (!(lz < Geo::T(A, 2) && cx < tg.c1[0] && cy < tg.c1[1] && cz < tg.c1[2])) return;
    const int ax = cell_origin<Geo>(A, rep, 0, cx) + o[0];
    const int ay = cell_origin<Geo>(A, rep, 1, cy) + o[1];
    const int az = cell_origin<Geo>(A, rep, 2, cz) + o[2];
    if constexpr (!Geo::fixed) {
        if (!(ax < cell_origin<Geo>(A, rep, 0, cx + 1) && ay < cell_origin<Geo>(A, rep, 1, cy + 1) &&
              az < cell_origin<Geo>(A, rep, 2, cz + 1)))
            return;
    }
    read_dispatch<LAT, E, Geo>(b, A, rep, T, win, tg, r, t, ax, ay, az, L);
}

template <int LAT, int E, class Geo>
__device__ __forceinline__ void tile_finish(const SweepArgs& A, const RepDev& rep, int r, uint32_t t, double beta,
                                            const Lds& T, uint8_t* win, const LaneState<E>& L, Stats& st)
{
    const int f = trial_finish<LAT, E, Geo>(A, rep, A.ws + rep.pad_off, T, win, r, t, beta, L);
    st.att += f & 1;
    st.acc += (f >> 1) & 1;
    st.tie += (f >> 2) & 1;
}

// Trials of basis sites b0 .. b0 + nb - 1 at the same offsets o, each lane in
// its own link cell.  One window serves them all: a lane's trial at b + 1
// reads within two conventional cells of its site, which no other cell's
// trial at b writes (the sites of two cells stay at least three cells apart
// on some axis), so the lane's own accepted swap, written back into the
// window, is the only change it can see.  (Needs every edge >= 4, so that no
// periodic image of a written site lies in that reach.)
template <int LAT, int E, class Geo>
__device__ __forceinline__ void tile_trials(const SweepArgs& A, const RepDev& rep, int r, const TileGeom& tg,
                                            int b0, int nb, const int (&o)[3], uint32_t t, double beta,
                                            const Lds& T, uint8_t* win, Stats& st)
{
    for (int j = 0; j < nb; ++j) {
        LaneState<E> L;
        tile_read<LAT, E, Geo>(A, rep, r, tg, b0 + j, o, t, T, win, L);
        tile_finish<LAT, E, Geo>(A, rep, r, t, beta, T, win, L, st);
    }
}

// The replica table is read-only during a launch: reading it through the
// constant address space (with a wave-uniform index) lets the compiler use
// scalar loads instead of per-lane ones.
__device__ __forceinline__ const RepDev& rep_of(const SweepArgs& A, int r)
{
    using CRep = const __attribute__((address_space(4))) RepDev;
    return *(const RepDev*)((CRep*)A.reps + r);
}

// Same for other tables a launch only reads (tile prefix sums, betas).
template <typename T>
__device__ __forceinline__ T ld_const(const T* p, int64_t i)
{
    using CT = const __attribute__((address_space(4))) T;
    return ((CT*)p)[i];
}

// The replica and tile of a loop step are the same in every lane; saying so
// lets the compiler read the replica's table through scalar loads.
__device__ __forceinline__ void uniform(int& r, int64_t& tile)
{
    r = __builtin_amdgcn_readfirstlane(r);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)tile);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)tile >> 32));
    tile = (int64_t)(((uint64_t)hi << 32) | lo);
}

// Tiles first, first + step, ... (< end) of a logical tile space for mini-step
// tau of sweep t.  With two window buffers the next tile's window streams into
// LDS while the current tile's trials run; with one, each window is staged in
// turn (half the LDS, so more workgroups per CU hide the latency instead).
// tile_of(i, r, tile) maps a logical index to (replica, tile of that replica);
// beta_of(r) gives the replica's inverse temperature.  Every thread calls this
// with the same arguments.
template <int LAT, int E, class Geo, int NBUF, typename TileOf, typename BetaOf>
__device__ void run_tiles(const SweepArgs& A, int64_t first, int64_t end, int64_t step, int tau, int nb, uint32_t t,
                          const Lds& T, uint8_t* win0, uint8_t* win1, TileOf tile_of, BetaOf beta_of, Stats& st,
                          int& r_stats)
{
    constexpr int m = kGeom[LAT].m;
    if (first >= end) return;
    auto offsets = [&](const RepDev& rep, int (&o)[3], int& b) {
        b = tau % m;
        const int rest = tau / m;
        o[0] = rest % rep.M[0];
        o[1] = (rest / rep.M[0]) % rep.M[1];
        o[2] = rest / (rep.M[0] * rep.M[1]);
    };
    if constexpr (NBUF == 1) {
        struct NoPlan {};
        [[maybe_unused]] std::conditional_t<Geo::fixed, StagePlan<LAT, Geo>, NoPlan> plan;
        for (int64_t i = first; i < end; i += step) {
            int r;
            int64_t tile;
            tile_of(i, r, tile);
            uniform(r, tile);
            const RepDev& rep = rep_of(A, r);
            if (tau >= rep.nA) continue;  // uniform across the block
            int o[3], b;
            offsets(rep, o, b);
            TileGeom tg;
            if (!tile_geometry<LAT, Geo>(A, rep, tile, o, tg)) continue;
            lds_barrier();  // every lane is done with the window of the previous tile
            const uint8_t* pad = A.ws + rep.pad_off;
            if constexpr (Geo::fixed) {
                constexpr int m = kGeom[LAT].m;
                using SP = decltype(plan);
                const int gx1 = (m * (tg.w0[0] + tg.n[0] + kHalo) + 15) & ~15;
                if (((gx1 - tg.gx0) >> 4) == SP::LPc && tg.n[1] == SP::WY && tg.n[2] == SP::WZ) {
                    plan.prepare(rep, r);
                    plan.stage_full(pad + ((int64_t)(tg.w0[2] + kHalo) * rep.prows + (tg.w0[1] + kHalo)) * rep.prow +
                                        tg.gx0,
                                    win0);
                } else {
                    stage_async<LAT, Geo>(A, rep, tg, pad, win0);
                }
            } else {
                stage_async<LAT, Geo>(A, rep, tg, pad, win0);
            }
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (r != r_stats) {
                flush_stats(A, r_stats, st);
                r_stats = r;
            }
            tile_trials<LAT, E, Geo>(A, rep, r, tg, b, nb, o, t, beta_of(r), T, win0, st);
        }
        return;
    }
    int r = 0, rn = 0;
    int64_t tile = 0, tilen = 0;
    tile_of(first, r, tile);
    uniform(r, tile);
    int o[3], b;
    TileGeom tg;
    bool have;
    constexpr bool dbl = true;
    {
        const RepDev& rep = rep_of(A, r);
        offsets(rep, o, b);
        have = tau < rep.nA && tile_geometry<LAT, Geo>(A, rep, tile, o, tg);
        if (have && dbl) stage_async<LAT, Geo>(A, rep, tg, A.ws + rep.pad_off, win0);
    }
    int k = 0;
    for (int64_t i = first; i < end; i += step, ++k) {
        const int64_t inext = i + step;
        int on[3] = {0, 0, 0}, bn = 0;
        TileGeom tgn;
        bool haven = false;
        if (inext < end) {
            tile_of(inext, rn, tilen);
            uniform(rn, tilen);
            const RepDev& repn = rep_of(A, rn);
            offsets(repn, on, bn);
            haven = tau < repn.nA && tile_geometry<LAT, Geo>(A, repn, tilen, on, tgn);
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();  // double buffering: window of tile i landed; both: lanes done with the buffer
        uint8_t* cur = win0;
        if (dbl) {
            cur = (k & 1) ? win1 : win0;
            if (haven) stage_async<LAT, Geo>(A, rep_of(A, rn), tgn, A.ws + rep_of(A, rn).pad_off, (k & 1) ? win0 : win1);
        } else if (have) {
            stage_async<LAT, Geo>(A, rep_of(A, r), tg, A.ws + rep_of(A, r).pad_off, win0);
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
        }
        if (have) {
            if (r != r_stats) {
                flush_stats(A, r_stats, st);
                r_stats = r;
            }
            tile_trials<LAT, E, Geo>(A, rep_of(A, r), r, tg, b, nb, o, t, beta_of(r), T, cur, st);
        }
        r = rn;
        tile = tilen;
        tg = tgn;
        have = haven;
        o[0] = on[0];
        o[1] = on[1];
        o[2] = on[2];
        b = bn;
    }
}

// ---------------------------------------------------------------------------
// Stream mode: one launch per mini-step g.  The logical tiles of all replicas
// (or of one replica in plain mode) are split into 8 contiguous chunks, one
// per XCD (hardware workgroup i runs on XCD i % 8); the workgroups of an XCD
// walk their chunk together with stride W, so neighbouring tiles -- which
// share halo rows -- are in flight on the same L2 at the same time.
// ---------------------------------------------------------------------------
template <int LAT, int E, class Geo, int NBUF>
__global__ __launch_bounds__(kBlock) void k_ministep(SweepArgs A)
{
    extern __shared__ __align__(16) uint8_t smem[];
    load_tables<LAT>(A, smem);
    const Lds T = lds_ptrs(A, smem);
    const int64_t total = A.only_rep >= 0 ? A.reps[A.only_rep].ntiles : A.tile_off[A.R];
    const int xcd = blockIdx.x % 8;
    const int64_t W = gridDim.x / 8;
    const int64_t chunk = (total + 7) / 8;
    const int64_t lo = xcd * chunk;
    const int64_t hi = min(lo + chunk, total);
    auto tile_of = [&](int64_t i, int& r, int64_t& tile) {
        if (A.only_rep >= 0) {
            r = A.only_rep;
            tile = i;
            return;
        }
        int a = 0, z = A.R - 1;  // last replica with tile_off[r] <= i
        while (a < z) {
            const int mid = (a + z + 1) >> 1;
            if (ld_const(A.tile_off, mid) <= i) a = mid; else z = mid - 1;
        }
        r = a;
        tile = i - ld_const(A.tile_off, a);
    };
    auto beta_of = [&](int r) { return ld_const(A.beta, r); };
    Stats st;
    int r_stats = -1;
    // a captured sweep reads its sweep index from the device counter
    const uint32_t t = A.sweep_counter ? *A.sweep_counter + A.first_sweep : A.first_sweep;
    run_tiles<LAT, E, Geo, NBUF>(A, lo + blockIdx.x / 8, hi, W, A.g, A.nb, t, T, smem + A.lds_win,
                           smem + A.lds_win + A.win_bytes, tile_of, beta_of, st, r_stats);
    flush_stats(A, r_stats, st);
}

// ---------------------------------------------------------------------------
// Row mode: one launch per group of mini-steps sharing the offsets (o_y, o_z)
// -- every o_x and basis site, M_x * m mini-steps.  A workgroup owns whole
// x-rows of link cells (T[1] x T[2] rows of every cell along x) and stages
// their window once: full padded x-rows, y and z within two cells of the
// active rows.  Within the group a trial depends only on trials of the same
// row (cells in other rows stay beyond the reach on y or z, since o_y and o_z
// are fixed), and there only on earlier offsets o_x; a workgroup barrier after
// each o_x orders them.  Accepted swaps go to HBM, to the window and to the
// window's x-images, so every later trial of the group reads them from LDS.
// A launch covers mini-steps g .. g + nb - 1 of one group.  MAXB: the largest
// workgroup the instantiation serves (1024 caps registers at 4 waves/SIMD).
// ---------------------------------------------------------------------------
// Trials of basis sites b0 .. b1 - 1 at one site of a lane's link cell, one
// code path per basis site (no merge of the sites' lane states).
template <int LAT, int E, class Geo, int B>
__device__ __forceinline__ void row_trials(int b0, int b1, const SweepArgs& A, const RepDev& rep, const Lds& T,
                                           uint8_t* win, const TileGeom& tg, int r, uint32_t t, double beta, int ax,
                                           int ay, int az, int64_t yz, Stats& st)
{
    if constexpr (B < kGeom[LAT].m) {
        if (B >= b0 && B < b1) {
            LaneState<E> L;
            trial_read<LAT, E, B, Geo>(A, rep, T, win, tg, r, t, ax, ay, az, L, yz);
            tile_finish<LAT, E, Geo>(A, rep, r, t, beta, T, win, L, st);
        }
        row_trials<LAT, E, Geo, B + 1>(b0, b1, A, rep, T, win, tg, r, t, beta, ax, ay, az, yz, st);
    }
}

// Basis-planar row segments a row group's trials can write: for a cell row
// whose active sites lie in row (ya, za), the active sites' own columns (every
// basis site) in that row, and for every partner direction the partner's
// column in the row it falls in.  Any other column of the rows around stays
// as it was staged.  Worked out at compile time from the shell-1 vectors.
struct WbSeg {
    int dy, dz, col;
};
struct WbPlan {
    int n;
    WbSeg seg[4 * 2 * kMaxZ1];
};

constexpr WbPlan make_wb_plan(const Geometry& G)
{
    WbPlan P{};
    P.n = 0;
    auto add = [&P](int dy, int dz, int col) {
        for (int i = 0; i < P.n; ++i)
            if (P.seg[i].dy == dy && P.seg[i].dz == dz && P.seg[i].col == col) return;
        P.seg[P.n].dy = dy;
        P.seg[P.n].dz = dz;
        P.seg[P.n].col = col;
        ++P.n;
    };
    for (int b = 0; b < G.m; ++b) {
        add(0, 0, b);
        for (int k = 0; k < G.Z[0]; ++k) {
            const Nb nb = nb_of(G, b, G.v[0][k][0], G.v[0][k][1], G.v[0][k][2]);
            add(nb.dy, nb.dz, nb.bt);
        }
    }
    return P;
}

// Copy the window row segments a row group's trials can have changed back to
// the padded copy: each segment (a basis column of a row within a partner's
// reach of the active row) to its own row and to its halo images when the row
// lies within H of a y or z face.  A whole column goes out, x-images included
// (the trials keep those current in the window).  No other workgroup of the
// launch changes these rows (their cells' active rows lie at least a cell edge
// away), so writing back bytes that did not change is harmless.  The T0 lanes
// of the cell row share its segments, 16 bytes per lane and item.
template <int LAT, class Geo>
__device__ __forceinline__ void rows_writeback(const SweepArgs& A, const RepDev& rep, const TileGeom& tg, int lx,
                                               int T0, int ya, int za, uint8_t* pad, const uint8_t* win)
{
    constexpr WbPlan W = make_wb_plan(kGeom[LAT]);
    constexpr int NS = W.n;
    const int LP = Geo::LP(A), WY = Geo::WY(A);
    const int cp = Geo::CP(rep), nc16 = cp >> 4;  // chunks of one basis column
    const int Ly = rep.L[1], Lz = rep.L[2];
    const int64_t prowp = rep.prowp, plane = (int64_t)rep.prows * prowp;
    // g lanes per segment, consecutive lanes on consecutive 16-byte chunks,
    // so a segment's addresses are worked out once per lane; with fewer lanes
    // than segments a lane takes segments lx, lx + T0, ...
    const int g = T0 / NS;
    int d = lx, dstep = T0, c0 = 0, cstep = 1;
    if (g > 0) {
        if (lx >= g * NS) return;
        d = lx / g;
        dstep = NS;
        c0 = lx - d * g;
        cstep = g;
    }
    for (; d < NS; d += dstep) {
        int dy = 0, dz = 0, col = 0;
#pragma unroll
        for (int i = 0; i < NS; ++i)
            if (i == d) {
                dy = W.seg[i].dy;
                dz = W.seg[i].dz;
                col = W.seg[i].col;
            }
        const int y = ya + dy, z = za + dz;  // in [-1, L]
        const int yr = y < 0 ? y + Ly : (y >= Ly ? y - Ly : y);
        const int zr = z < 0 ? z + Lz : (z >= Lz ? z - Lz : z);
        const int yi = yr < kHalo ? yr + Ly : (yr >= Ly - kHalo ? yr - Ly : yr);  // image, or yr itself
        const int zi = zr < kHalo ? zr + Lz : (zr >= Lz - kHalo ? zr - Lz : zr);
        const uint8_t* src = win + ((z - tg.w0[2]) * WY + (y - tg.w0[1])) * LP + col * cp + 16 * c0;
        uint8_t* dst = pad + (zr + kHalo) * plane + (yr + kHalo) * prowp + col * cp + 16 * c0;
        const int64_t ddy = (int64_t)(yi - yr) * prowp, ddz = (int64_t)(zi - zr) * plane;  // images (0: none)
        for (int c = c0; c < nc16; c += cstep) {
            const uint4 v = *(const uint4*)src;
            *(uint4*)dst = v;
            if (ddy) *(uint4*)(dst + ddy) = v;
            if (ddz) *(uint4*)(dst + ddz) = v;
            if (ddy && ddz) *(uint4*)(dst + ddy + ddz) = v;
            src += 16 * cstep;
            dst += 16 * cstep;
        }
    }
}

template <int LAT, int E, class Geo, int MAXB>
__global__ __launch_bounds__(MAXB) void k_rows(SweepArgs A)
{
    constexpr int m = kGeom[LAT].m;
    extern __shared__ __align__(16) uint8_t smem[];
    load_tables<LAT>(A, smem);
    const Lds T = lds_ptrs(A, smem);
    uint8_t* win = smem + A.lds_win;
    const int64_t total = ld_const(A.tile_off, A.R);  // row groups of all replicas
    const int xcd = blockIdx.x % 8;
    const int64_t W = gridDim.x / 8;
    const int64_t chunk = (total + 7) / 8;
    const int64_t lo = xcd * chunk;
    const int64_t hi = min(lo + chunk, total);
    const int l = threadIdx.x;
    const int T0 = Geo::T(A, 0), T1 = Geo::T(A, 1), T2 = Geo::T(A, 2);
    const int lx = l % T0, ly = (l / T0) % T1, lz = l / (T0 * T1);
    const uint32_t t = A.sweep_counter ? *A.sweep_counter + A.first_sweep : A.first_sweep;
    Stats st;
    int r_stats = -1;
    for (int64_t i = lo + blockIdx.x / 8; i < hi; i += W) {
        int a = 0, z = A.R - 1;  // last replica with tile_off[r] <= i
        while (a < z) {
            const int mid = (a + z + 1) >> 1;
            if (ld_const(A.tile_off, mid) <= i) a = mid; else z = mid - 1;
        }
        int r = a;
        int64_t grp = i - ld_const(A.tile_off, a);
        uniform(r, grp);
        const RepDev& rep = rep_of(A, r);
        int g0 = A.g, gn = A.nb;
        if (A.gq >= 0) {
            // this replica's q-th (o_y, o_z) group, every offset o_x and basis site
            if (A.gq >= rep.M[1] * rep.M[2]) continue;
            gn = m * rep.M[0];
            g0 = A.gq * gn;
        }
        if (g0 >= rep.nA) continue;
        const int b0 = g0 % m, rest = g0 / m;
        const int ox0 = rest % rep.M[0];
        const int oy = (rest / rep.M[0]) % rep.M[1], oz = rest / (rep.M[0] * rep.M[1]);
        const int gy = (int)(grp % rep.rg[0]), gz = (int)(grp / rep.rg[0]);
        TileGeom tg;
        tg.c0[0] = 0;
        tg.c1[0] = rep.nc[0];
        tg.c0[1] = gy * T1;
        tg.c1[1] = min(tg.c0[1] + T1, rep.nc[1]);
        tg.c0[2] = gz * T2;
        tg.c1[2] = min(tg.c0[2] + T2, rep.nc[2]);
        if (oy >= rep.emin[1] || oz >= rep.emin[2]) {
            // uneven partitions: offsets past the shorter cells leave some row
            // groups without an active cell row; skip them before staging
            bool any_y = false, any_z = false;
            for (int c = tg.c0[1]; c < tg.c1[1]; ++c)
                any_y |= cell_origin<Geo>(A, rep, 1, c + 1) - cell_origin<Geo>(A, rep, 1, c) > oy;
            for (int c = tg.c0[2]; c < tg.c1[2]; ++c)
                any_z |= cell_origin<Geo>(A, rep, 2, c + 1) - cell_origin<Geo>(A, rep, 2, c) > oz;
            if (!(any_y && any_z)) continue;
        }
        tg.w0[0] = -kHalo;
        tg.n[0] = rep.L[0] + 2 * kHalo;
        tg.gx0 = 0;
        const int oo[3] = {0, oy, oz};
#pragma unroll
        for (int ax = 1; ax < 3; ++ax) {
            tg.w0[ax] = cell_origin<Geo>(A, rep, ax, tg.c0[ax]) + oo[ax] - kHalo;
            const int w1 = min(cell_origin<Geo>(A, rep, ax, tg.c1[ax] - 1) + oo[ax] + kHalo + 1, rep.L[ax] + kHalo);
            tg.n[ax] = w1 - tg.w0[ax];
        }
        if (tg.n[1] <= 0 || tg.n[2] <= 0) continue;
        lds_barrier();  // every lane is done with the previous window
        stage_async<LAT, Geo>(A, rep, tg, A.ws + rep.pad_off, win);
        // this lane's cell while the loads fly
        const int cx = lx, cy = tg.c0[1] + ly, cz = tg.c0[2] + lz;
        const bool row_in = lz < T2 && cy < tg.c1[1] && cz < tg.c1[2];
        const bool in = row_in && cx < tg.c1[0];
        int x0 = 0, ex = 0, y0 = 0, ey = 0, z0 = 0, ez = 0;
        if (row_in) {
            y0 = cell_origin<Geo>(A, rep, 1, cy);
            ey = cell_origin<Geo>(A, rep, 1, cy + 1) - y0;
            z0 = cell_origin<Geo>(A, rep, 2, cz);
            ez = cell_origin<Geo>(A, rep, 2, cz + 1) - z0;
        }
        if (in) {
            x0 = cell_origin<Geo>(A, rep, 0, cx);
            ex = cell_origin<Geo>(A, rep, 0, cx + 1) - x0;
        }
        // the cell row has active sites at (o_y, o_z)
        const bool row_yz = row_in && oy < ey && oz < ez;
        const bool yz = in && row_yz;
        const double beta = ld_const(A.beta, r);
        const int64_t yz_site = (int64_t)m * rep.L[0] * ((int64_t)(y0 + oy) + (int64_t)rep.L[1] * (z0 + oz));
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (r != r_stats) {
            flush_stats_block(A, r_stats, st);
            r_stats = r;
        }
        int tau = g0, b = b0, ox = ox0;
        const int tau1 = g0 + gn;
        while (true) {
            const int nbb = min(m - b, tau1 - tau);
            if (yz && ox < ex)
                row_trials<LAT, E, Geo, 0>(b, b + nbb, A, rep, T, win, tg, r, t, beta, x0 + ox, y0 + oy, z0 + oz, yz_site, st);
            tau += nbb;
            if (tau >= tau1) break;
            b = 0;
            ++ox;
            __syncthreads();  // the next offset's trials read what this one wrote
        }
        __syncthreads();  // every trial's window writes are visible
        if (row_yz) rows_writeback<LAT, Geo>(A, rep, tg, lx, T0, y0 + oy, z0 + oz, A.ws + rep.pad_off, win);
    }
    flush_stats_block(A, r_stats, st);
}

// ---------------------------------------------------------------------------
// Persistent mode: one workgroup per replica runs every sweep and mini-step;
// block barriers order the mini-steps (all writes of a replica come from its
// own workgroup, and a barrier makes them visible to its later loads).
// ---------------------------------------------------------------------------
template <int LAT, int E, class Geo>
__global__ __launch_bounds__(kBlock) void k_persistent(SweepArgs A)
{
    extern __shared__ __align__(16) uint8_t smem[];
    const int r = blockIdx.x;
    const RepDev& rep = rep_of(A, r);
    load_tables<LAT>(A, smem);
    const Lds T = lds_ptrs(A, smem);
    const uint32_t first = A.sweep_counter ? *A.sweep_counter : A.first_sweep;
    auto tile_of = [&](int64_t i, int& rr, int64_t& tile) {
        rr = r;
        tile = i;
    };
    Stats st;
    int r_stats = r;
    const int tau_end = min(A.tau_end, rep.nA);
    for (int js = 0; js < A.n_sweeps; ++js) {
        const uint32_t t = first + (uint32_t)js;
        const double beta = ld_const(A.beta, (int64_t)js * A.beta_stride + r);
        auto beta_of = [&](int) { return beta; };
        for (int tau = A.tau_begin; tau < tau_end;) {
            // mini-steps of consecutive basis sites at one offset share a window
            const int nb = min(A.nb - tau % A.nb, tau_end - tau);
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();  // the previous mini-step's writes are visible to every wave
            run_tiles<LAT, E, Geo, 1>(A, 0, rep.ntiles, 1, tau, nb, t, T, smem + A.lds_win,
                                   smem + A.lds_win + A.win_bytes, tile_of, beta_of, st, r_stats);
            tau += nb;
        }
    }
    flush_stats(A, r_stats, st);
}

__global__ void k_advance_counter(uint32_t* counter, uint32_t n)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *counter += n;
}

// Natural layout -> padded copy.  A workgroup fills whole padded rows
// (halo rows and columns included: each padded row is the natural row at the
// wrapped y, z, each byte the site at the wrapped x), a thread one dword of
// the row at a time; bytes past a column's L0 + 2H sites stay 0.
// One word of a padded row byte by byte (halo columns wrap to the far side).
template <int M, bool PLANAR>
__device__ __forceinline__ uint32_t pack_word(const RepDev& rep, const uint8_t* src, int w, int L0, int F)
{
    uint32_t v = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int j = 4 * w + i;
        const int b = PLANAR ? j / rep.cp : j % M;
        int x = (PLANAR ? j - b * rep.cp : j / M) - kHalo;
        if (b < M && x < L0 + kHalo) {
            x += x < 0 ? L0 : (x >= L0 ? -L0 : 0);
            v |= (uint32_t)(src[M * x + b] * F) << (8 * i);
        }
    }
    return v;
}

template <int M, bool PLANAR>
__global__ void k_pack(const uint8_t* occ, uint8_t* ws, const RepDev* reps, int r, int F)
{
    const RepDev& rep = reps[r < 0 ? (int)blockIdx.y : r];  // r < 0: one replica per grid row
    uint8_t* pad = ws + rep.pad_off;
    const uint8_t* o = occ + rep.occ_off;
    const int L0 = rep.L[0], L1 = rep.L[1], L2 = rep.L[2];
    const int pitch = PLANAR ? rep.prowp : rep.prow;
    const int nrow = rep.prows * (L2 + 2 * kHalo);
    const int words = pitch >> 2;
    if (M == 2 && PLANAR && (rep.cp >> 4) <= (int)blockDim.x) {
        // Two basis sites, planar rows of 16-byte aligned columns: a thread
        // takes 16 cells of a row (x0 = 16 j - 2 .. x0 + 15, 32 natural bytes
        // read once as 8 aligned words, or 9 shifted by 2 bytes when the row
        // starts 2 bytes past a word boundary) and writes both basis columns'
        // 16 bytes with one store each; blocks that wrap or pass the row's
        // end, and the bytes past the two columns, go word by word
        const int nblk = rep.cp >> 4, tail0 = 2 * (rep.cp >> 2);
        const int rows_per = (int)blockDim.x / nblk;  // at least one row per pass
        const int lr = (int)threadIdx.x / nblk, j = (int)threadIdx.x - lr * nblk;
        for (int row0 = blockIdx.x * rows_per; row0 < nrow; row0 += gridDim.x * rows_per) {
            const int row = row0 + lr;
            if (lr < rows_per && row < nrow) {
                const int yp = row % rep.prows, zp = row / rep.prows;
                int y = yp - kHalo, z = zp - kHalo;
                y += y < 0 ? L1 : (y >= L1 ? -L1 : 0);
                z += z < 0 ? L2 : (z >= L2 ? -L2 : 0);
                const uint8_t* src = o + (int64_t)M * L0 * (y + (int64_t)L1 * z);
                uint32_t* dst = (uint32_t*)(pad + (int64_t)row * pitch);
                const int sh = (int)((uintptr_t)src & 3);  // 0 or 2
                const int x0 = 16 * j - kHalo;
                if (x0 >= 0 && x0 + 16 + (sh >> 1) <= L0) {
                    const uint32_t* s32 = (const uint32_t*)(src + 2 * x0 - sh);
                    uint32_t d[9];
#pragma unroll
                    for (int i = 0; i < 8; ++i) d[i] = s32[i];
                    if (sh) {
                        d[8] = s32[8];
#pragma unroll
                        for (int i = 0; i < 8; ++i) d[i] = __builtin_amdgcn_alignbyte(d[i + 1], d[i], (uint32_t)sh);
                    }
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        uint4 v;
                        v.x = __builtin_amdgcn_perm(d[1], d[0], b ? 0x07050301u : 0x06040200u) * (uint32_t)F;
                        v.y = __builtin_amdgcn_perm(d[3], d[2], b ? 0x07050301u : 0x06040200u) * (uint32_t)F;
                        v.z = __builtin_amdgcn_perm(d[5], d[4], b ? 0x07050301u : 0x06040200u) * (uint32_t)F;
                        v.w = __builtin_amdgcn_perm(d[7], d[6], b ? 0x07050301u : 0x06040200u) * (uint32_t)F;
                        *(uint4*)(dst + b * (rep.cp >> 2) + 4 * j) = v;
                    }
                } else {
#pragma unroll
                    for (int b = 0; b < 2; ++b)
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            const int w = b * (rep.cp >> 2) + 4 * j + t;
                            dst[w] = pack_word<M, PLANAR>(rep, src, w, L0, F);
                        }
                }
                if (j == 0)
                    for (int w = tail0; w < words; ++w) dst[w] = 0u;
            }
        }
        return;
    }
    for (int row = blockIdx.x; row < nrow; row += gridDim.x) {
        const int yp = row % rep.prows, zp = row / rep.prows;
        int y = yp - kHalo, z = zp - kHalo;
        y += y < 0 ? L1 : (y >= L1 ? -L1 : 0);
        z += z < 0 ? L2 : (z >= L2 ? -L2 : 0);
        const uint8_t* src = o + (int64_t)M * L0 * (y + (int64_t)L1 * z);
        uint32_t* dst = (uint32_t*)(pad + (int64_t)row * pitch);
        // two basis sites, planar rows: a word of basis b at x .. x + 3 (no
        // wrap) is bytes b, b + 2, b + 4, b + 6 of the natural row from 2 x,
        // two natural words (or, in a row that starts 2 bytes past a word
        // boundary -- odd L0 -- three aligned words shifted by 2 bytes), and
        // times F byte by byte (every F * species < 256, so no carry crosses
        // a byte)
        const int sh = (int)((uintptr_t)src & 3);  // 0 or 2: natural rows hold an even number of bytes
        const bool fast = M == 2 && PLANAR && (sh & 1) == 0;
        const int cpw = rep.cp >> 2;
        for (int w = threadIdx.x; w < words; w += blockDim.x) {
            if (fast) {
                const int b = w >= cpw ? 1 : 0;
                const int xw = 4 * (w - b * cpw) - kHalo;
                // every byte read lies in this natural row
                if (xw >= 0 && xw + 3 + (sh >> 1) < L0) {
                    const uint32_t* s32 = (const uint32_t*)(src + 2 * xw - sh);
                    uint32_t lo = s32[0], hi = s32[1];
                    if (sh) {
                        const uint32_t h2 = s32[2];
                        lo = __builtin_amdgcn_alignbyte(hi, lo, (uint32_t)sh);
                        hi = __builtin_amdgcn_alignbyte(h2, hi, (uint32_t)sh);
                    }
                    const uint32_t v = __builtin_amdgcn_perm(hi, lo, b ? 0x07050301u : 0x06040200u);
                    dst[w] = v * (uint32_t)F;
                    continue;
                }
            }
            dst[w] = pack_word<M, PLANAR>(rep, src, w, L0, F);
        }
    }
}

// Padded copy interior -> natural layout: a workgroup per natural row, a
// thread per site byte.
template <int M, bool PLANAR>
__global__ void k_unpack(uint8_t* occ, const uint8_t* ws, const RepDev* reps, int r, int F)
{
    const RepDev& rep = reps[r < 0 ? (int)blockIdx.y : r];  // r < 0: one replica per grid row
    const uint8_t* pad = ws + rep.pad_off;
    uint8_t* o = occ + rep.occ_off;
    const int L0 = rep.L[0], L1 = rep.L[1], L2 = rep.L[2];
    const int pitch = PLANAR ? rep.prowp : rep.prow;
    const int n = M * L0;
    for (int row = blockIdx.x; row < L1 * L2; row += gridDim.x) {
        const int y = row % L1, z = row / L1;
        const uint8_t* src = pad + ((int64_t)(z + kHalo) * rep.prows + (y + kHalo)) * pitch;
        uint8_t* dst = o + (int64_t)n * row;
        // two basis sites, planar rows, F = 8, rows of a whole number of
        // words: natural word w (x = 2w, 2w + 1, both basis sites)
        // interleaves two bytes of each basis column, taken from the aligned
        // word holding them (x + H is even, so the pair never straddles one)
        if (M == 2 && PLANAR && F == 8 && (n & 3) == 0 && ((uintptr_t)dst & 3) == 0 && ((uintptr_t)src & 3) == 0) {
            uint32_t* d32 = (uint32_t*)dst;
            const int nw = n >> 2;
            // a thread's two words load before either is stored
            for (int w0 = threadIdx.x; w0 < nw; w0 += 2 * blockDim.x) {
                uint32_t a[2] = {0u, 0u}, bb[2] = {0u, 0u};
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int w = w0 + u * (int)blockDim.x;
                    if (w < nw) {
                        const int c0 = kHalo + 2 * w, c1 = rep.cp + kHalo + 2 * w;  // bytes of (2w, b = 0), (2w, b = 1)
                        a[u] = *(const uint32_t*)(src + (c0 & ~3));
                        bb[u] = *(const uint32_t*)(src + (c1 & ~3));
                    }
                }
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int w = w0 + u * (int)blockDim.x;
                    if (w >= nw) continue;
                    const uint32_t o = (uint32_t)((kHalo + 2 * w) & 3);  // 0 or 2, the same in both columns (cp is a multiple of 16)
                    const uint32_t sel = o | ((4 + o) << 8) | ((o + 1) << 16) | ((5 + o) << 24);
                    d32[w] = (__builtin_amdgcn_perm(bb[u], a[u], sel) >> 3) & 0x1F1F1F1Fu;
                }
            }
            continue;
        }
        // rows of 2 mod 4 bytes (odd L0), every other one starting 2 bytes
        // past a word boundary: the words from the first aligned byte (x =
        // x0 + 2w, x0 + 1 + 2w), each column's byte pair taken from the two
        // aligned words around it; the bytes before and after, one by one
        if (M == 2 && PLANAR && F == 8 && (n & 3) == 2 && ((uintptr_t)dst & 1) == 0 && ((uintptr_t)src & 3) == 0) {
            const int pos = (int)((4 - ((uintptr_t)dst & 3)) & 3);  // 0 or 2 bytes before the first word
            const int nw = (n - pos) >> 2, x0 = pos >> 1;
            uint32_t* d32 = (uint32_t*)(dst + pos);
            for (int w = threadIdx.x; w < nw; w += blockDim.x) {
                const int c0 = kHalo + x0 + 2 * w, c1 = rep.cp + c0;  // bytes of (x, b = 0), (x, b = 1)
                const uint32_t* a32 = (const uint32_t*)(src + (c0 & ~3));
                const uint32_t* b32 = (const uint32_t*)(src + (c1 & ~3));
                const uint32_t pa = __builtin_amdgcn_alignbyte(a32[1], a32[0], (uint32_t)(c0 & 3));
                const uint32_t pb = __builtin_amdgcn_alignbyte(b32[1], b32[0], (uint32_t)(c1 & 3));
                d32[w] = (__builtin_amdgcn_perm(pb, pa, 0x05010400u) >> 3) & 0x1F1F1F1Fu;
            }
            const int tail = pos + 4 * nw;
            for (int j = threadIdx.x; j < n - tail + pos; j += blockDim.x) {
                const int jj = j < pos ? j : tail + (j - pos);
                const int x = jj >> 1, b = jj & 1;
                dst[jj] = (uint8_t)species_of(src[row_byte<PLANAR>(rep, M, x, b)], F);
            }
            continue;
        }
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            const int x = j / M, b = j - x * M;
            dst[j] = (uint8_t)species_of(src[row_byte<PLANAR>(rep, M, x, b)], F);
        }
    }
}

__global__ void k_validate(const uint8_t* occ, int64_t n, int K, int32_t* bad)
{
    int found = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        found |= occ[i] >= K;
    if (__ballot(found) && (threadIdx.x & 63) == 0) atomicOr(bad, 1);
}

__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// Pair counts C[cfg][s][k][l] on the natural layout, periodic wrap through
// per-site wrapped coordinates.  One thread per conventional cell (all its
// basis sites), shells processed one after another; per-lane counts kept in
// 16-bit fields (<= 24 per site, <= 2048 sites per lane between flushes),
// then wave-reduced and added with 64-bit atomics.  (Pair numbers n_m^{pp'}
// of the EPI features, Methods "The EPI and qSRO model".)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int LAT, int KP>
__global__ __launch_bounds__(kBlock) void k_pair_counts(const uint8_t* occ, int64_t N, int L0, int L1, int L2,
                                                        int K, int S, int cells_per_block, int64_t* counts)
{
    constexpr Geometry G = kGeom[LAT];
    constexpr int m = G.m;
    const int cfg = blockIdx.y;
    const uint8_t* o = occ + (int64_t)cfg * N;
    const int64_t ncell = (int64_t)L0 * L1 * L2;
    const int64_t cb = (int64_t)blockIdx.x * cells_per_block;
    const int64_t ce = min(cb + cells_per_block, ncell);
    const int64_t plane = (int64_t)L0 * L1;
#pragma unroll
    for (int s = 0; s < kMaxShells; ++s) {
        if (s >= S) break;
        uint32_t acc[KP][KP / 2];
#pragma unroll
        for (int k = 0; k < KP; ++k)
#pragma unroll
            for (int j = 0; j < KP / 2; ++j) acc[k][j] = 0;
        for (int64_t c = cb + threadIdx.x; c < ce; c += blockDim.x) {
            const int x = (int)(c % L0);
            const int64_t cr = c / L0;
            const int y = (int)(cr % L1);
            const int z = (int)(cr / L1);
            int64_t X[5], Y[5], Z[5];
#pragma unroll
            for (int d = -2; d <= 2; ++d) {
                int xx = x + d, yy = y + d, zz = z + d;
                xx += xx < 0 ? L0 : (xx >= L0 ? -L0 : 0);
                yy += yy < 0 ? L1 : (yy >= L1 ? -L1 : 0);
                zz += zz < 0 ? L2 : (zz >= L2 ? -L2 : 0);
                X[d + 2] = xx;
                Y[d + 2] = (int64_t)yy * L0;
                Z[d + 2] = (int64_t)zz * plane;
            }
#pragma unroll
            for (int b = 0; b < m; ++b) {
                const int sig = o[m * c + b];
                uint64_t n = 0;
#pragma unroll
                for (int i = 0; i < G.Z[s]; ++i) {
                    const Nb nb = nb_of(G, b, G.v[s][i][0], G.v[s][i][1], G.v[s][i][2]);
                    const int64_t j = (int64_t)m * (X[nb.dx + 2] + Y[nb.dy + 2] + Z[nb.dz + 2]) + nb.bt;
                    n += (uint64_t)1 << (8 * o[j]);
                }
#pragma unroll
                for (int k = 0; k < KP; ++k) {
                    const uint32_t mask = sig == k ? 0xFFFFFFFFu : 0u;
#pragma unroll
                    for (int jj = 0; jj < KP / 2; ++jj) {
                        const uint32_t w = (uint32_t)((n >> (16 * jj)) & 0xFF) |
                                           ((uint32_t)((n >> (16 * jj + 8)) & 0xFF) << 16);
                        acc[k][jj] += w & mask;
                    }
                }
            }
        }
        int64_t* Cs = counts + ((int64_t)cfg * S + s) * K * K;
#pragma unroll
        for (int k = 0; k < KP; ++k) {
#pragma unroll
            for (int jj = 0; jj < KP / 2; ++jj) {
                const uint32_t lo = wave_sum(acc[k][jj] & 0xFFFFu);
                const uint32_t hi = wave_sum(acc[k][jj] >> 16);
                if ((threadIdx.x & 63) == 0 && k < K) {
                    if (2 * jj < K && lo)
                        atomicAdd((unsigned long long*)&Cs[k * K + 2 * jj], (unsigned long long)lo);
                    if (2 * jj + 1 < K && hi)
                        atomicAdd((unsigned long long*)&Cs[k * K + 2 * jj + 1], (unsigned long long)hi);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Pair counts of up to 4 species through LDS tiles: a block stages TX x TY x
// 16 conventional cells plus a 2-cell periodic halo of one configuration;
// lane (x, y) walks the 16 cells along z, forms the packed neighbour
// histogram of each site per shell over one direction d of every +-d pair
// (one byte read and one shift-add per neighbour, offsets fixed at compile
// time) and adds it to 16-bit fields of the row of the site's species.  These
// half-shell counts H give the directed counts as C[k][l] = H[k][l] +
// H[l][k]: the pairs along -d from species k to l are those along +d from l
// to k.  tiles_per_block keeps every field below 2^16 between flushes.
// ---------------------------------------------------------------------------
template <int LAT, int TX>
__global__ __launch_bounds__(kBlock) void k_pair_counts_tiled(const uint8_t* occ, int64_t N, int L0, int L1, int L2,
                                                              int K, int S, int tiles_per_block, int64_t* counts)
{
    constexpr Geometry G = kGeom[LAT];
    constexpr int m = G.m;
    constexpr int TY = kBlock / TX, TZ = 16;
    constexpr int WX = TX + 2 * kHalo, WY = TY + 2 * kHalo, WZ = TZ + 2 * kHalo;
    constexpr int LP = WX * m, PL = LP * WY;
    __shared__ __align__(16) uint8_t win[PL * WZ];
    const uint8_t* o = occ + (int64_t)blockIdx.y * N;
    const int ntx = (L0 + TX - 1) / TX, nty = (L1 + TY - 1) / TY, ntz = (L2 + TZ - 1) / TZ;
    const int64_t ntiles = (int64_t)ntx * nty * ntz;
    const int64_t t0 = (int64_t)blockIdx.x * tiles_per_block;
    const int64_t t1 = min(t0 + (int64_t)tiles_per_block, ntiles);
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    auto wrap = [](int v, int L) {
        v += v < 0 ? L : 0;
        v -= v >= L ? L : 0;
        return v >= L ? v % L : v;  // only lattices narrower than a tile wrap twice
    };
    uint32_t acc[4][kMaxShells][2];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int s = 0; s < kMaxShells; ++s) acc[k][s][0] = acc[k][s][1] = 0;
    for (int64_t ti = t0; ti < t1; ++ti) {
        const int tx = (int)(ti % ntx);
        const int64_t tr = ti / ntx;
        const int ty = (int)(tr % nty), tz = (int)(tr / nty);
        const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
        __syncthreads();  // every lane is done with the previous tile
        if constexpr (TX >= 64) {
            // a wave per window row: its wrapped y, z and base address are
            // wave-uniform, a lane wraps only its own x
            const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
            for (int rr = wave; rr < WY * WZ; rr += kBlock / 64) {
                const int wy = rr % WY, wz = rr / WY;
                const int y = wrap(y0 + wy - kHalo, L1), z = wrap(z0 + wz - kHalo, L2);
                const uint8_t* row = o + (int64_t)m * L0 * (y + (int64_t)L1 * z);
                uint8_t* d = win + (wz * WY + wy) * LP;
                for (int wx = lane; wx < WX; wx += 64) {
                    const int x = wrap(x0 + wx - kHalo, L0);
                    if constexpr (m == 2) *(uint16_t*)(d + 2 * wx) = *(const uint16_t*)(row + 2 * x);
                    else *(uint32_t*)(d + 4 * wx) = *(const uint32_t*)(row + 4 * x);
                }
            }
        } else {
            for (int c = threadIdx.x; c < WX * WY * WZ; c += blockDim.x) {
                const int wx = c % WX, wr = c / WX, wy = wr % WY, wz = wr / WY;
                const int x = wrap(x0 + wx - kHalo, L0), y = wrap(y0 + wy - kHalo, L1), z = wrap(z0 + wz - kHalo, L2);
                const int64_t cell = x + (int64_t)L0 * (y + (int64_t)L1 * z);
                uint8_t* d = win + (wz * WY + wy) * LP + wx * m;
                if constexpr (m == 2) *(uint16_t*)d = *(const uint16_t*)(o + 2 * cell);
                else *(uint32_t*)d = *(const uint32_t*)(o + 4 * cell);
            }
        }
        __syncthreads();
        if (x0 + lx >= L0 || y0 + ly >= L1) continue;
        for (int lz = 0; lz < TZ && z0 + lz < L2; ++lz) {
#pragma unroll
            for (int b = 0; b < m; ++b) {
                const int base = ((lz + kHalo) * WY + (ly + kHalo)) * LP + (lx + kHalo) * m + b;
                const int sig = win[base];
#pragma unroll
                for (int s = 0; s < kMaxShells; ++s) {
                    if (s < S) {
                        // one direction of every +-d pair: these half-shell
                        // counts H give C[k][l] = H[k][l] + H[l][k] exactly
                        constexpr int kHalfZ = kMaxZ / 2;
                        uint32_t v[kHalfZ];
#pragma unroll
                        for (int n = 0; n < G.Z[s] / 2; ++n) {
                            const Nb nb = nb_of(G, b, G.v[s][n][0], G.v[s][n][1], G.v[s][n][2]);
                            v[n] = win[base + nb.dz * PL + nb.dy * LP + m * nb.dx + (nb.bt - b)];
                        }
                        uint32_t h = 0;
#pragma unroll
                        for (int n = 0; n < G.Z[s] / 2; ++n) h += 1u << (8 * v[n]);
                        // 8-bit fields (<= 24 each) -> two words of 16-bit fields
                        const uint32_t lo = (h & 0xFFu) | ((h & 0xFF00u) << 8);
                        const uint32_t hi = ((h >> 16) & 0xFFu) | ((h >> 8) & 0xFF0000u);
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            acc[k][s][0] += sig == k ? lo : 0u;
                            acc[k][s][1] += sig == k ? hi : 0u;
                        }
                    }
                }
            }
        }
    }
    int64_t* C = counts + (int64_t)blockIdx.y * S * K * K;
#pragma unroll
    for (int s = 0; s < kMaxShells; ++s) {
        if (s >= S) continue;
        // the wave's half-shell counts H[k][l], then C[k][l] and C[l][k] each
        // gain H[k][l] + H[l][k] in one atomic
        uint32_t H[4][4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                H[k][2 * j] = k < K ? wave_sum(acc[k][s][j] & 0xFFFFu) : 0u;
                H[k][2 * j + 1] = k < K ? wave_sum(acc[k][s][j] >> 16) : 0u;
            }
        if ((threadIdx.x & 63) == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int l = k; l < 4; ++l) {
                    const uint32_t c = H[k][l] + H[l][k];
                    if (l >= K || c == 0) continue;
                    atomicAdd((unsigned long long*)&C[(s * K + k) * K + l], (unsigned long long)c);
                    if (l != k) atomicAdd((unsigned long long*)&C[(s * K + l) * K + k], (unsigned long long)c);
                }
        }
    }
}

// ---------------------------------------------------------------------------
// Pair counts of up to 5 species over slabs of whole x-rows: a workgroup owns
// kSlabY consecutive rows (all of x) and a run of planes along z, and walks
// the planes with a ring of 4 window planes in LDS: planes z .. z + 2 are
// read while plane z + 3 comes in through registers.  Each site counts one
// direction of every +-d pair, the one with d_z > 0 (or d_z = 0 and d_y > 0,
// or d_z = d_y = 0 and d_x > 0), so its neighbours lie in planes z .. z + 2,
// rows y - 2 .. y + 2 and cells x - 2 .. x + 2; as in the tiled kernel these
// half-shell counts H give C[k][l] = H[k][l] + H[l][k].  Every byte of the
// lattice is read (kSlabY + 4) / kSlabY times plus the ring's two extra planes
// per run, instead of the tiles' 2-3x halo re-reads.  Planes come in by
// LDS-direct loads while the previous plane is counted, then are scaled in
// place to F * species, F = 8 for up to 4 species and 6 for 5 (a neighbour
// costs one LDS byte read and one shift-add into F-bit fields, each at most
// 12); a site's histogram goes into 16-bit fields of its species'
// accumulators by 24-bit multiply-adds with a 0/1 factor.
// ---------------------------------------------------------------------------
constexpr int kSlabY = 8;
constexpr int kSlabBlock = 512;

// Positive half of shell s of a basis-b site as (dz, dy, dx, bt), in shell order.
constexpr bool positive(const int (&v)[3]) { return v[2] > 0 || (v[2] == 0 && (v[1] > 0 || (v[1] == 0 && v[0] > 0))); }

template <int LAT, int KF>
__global__ __launch_bounds__(kSlabBlock) void k_pair_counts_slab(const uint8_t* occ, int64_t N, int L0, int L1, int L2,
                                                               int K, int S, int ZC, int pitch, int64_t* counts)
{
    static_assert(KF == 4 || KF == 5, "up to 4 species in 8-bit fields, 5 in 6-bit fields");
    constexpr int F = KF == 5 ? 6 : 8;  // field width of the site histograms
    constexpr int NWD = (KF + 1) / 2;   // words of 16-bit fields per species accumulator
    constexpr Geometry G = kGeom[LAT];
    constexpr int m = G.m;
    constexpr int NR = kSlabY + 4;
    extern __shared__ __align__(16) uint8_t win[];  // 4 planes x NR rows x pitch
    const int plane_bytes = NR * pitch;
    const uint8_t* o = occ + (int64_t)blockIdx.z * N;
    const int y0 = blockIdx.x * kSlabY;
    const int z0 = blockIdx.y * ZC, z1 = min(z0 + ZC, L2);
    const int rowd = (L0 * m) >> 2;  // dwords of a natural row
    constexpr int hd = m / 2;        // dwords of a 2-cell halo
    const int nd = rowd + 2 * hd;    // dwords of a window row: cells -2 .. L0 + 1
    const int nitems = NR * nd;
    auto wrap = [](int v, int L) {
        v %= L;
        return v < 0 ? v + L : v;
    };
    // plane z into ring slot `slot`: window row rr is natural row y0 - 2 + rr
    // (wrapped), dword j of it the natural dword of cell 2 j / m - 2 (wrapped);
    // copied straight into LDS, a wave per window row, 64 dwords per load
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    auto stage = [&](int z, int slot) {
        const int zw = wrap(z, L2);
        uint8_t* base = win + slot * plane_bytes;
        for (int rr = wave; rr < NR; rr += kSlabBlock / 64) {
            const int y = wrap(y0 - kHalo + rr, L1);
            const uint32_t* row = (const uint32_t*)(o + (int64_t)m * L0 * (y + (int64_t)L1 * zw));
            for (int cb = 0; cb < nd; cb += 64) {
                const int j = cb + lane;
                if (j < nd) {
                    const int jj = j < hd ? rowd - hd + j : (j < hd + rowd ? j - hd : j - hd - rowd);
                    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(row + jj),
                                                     (__attribute__((address_space(3))) void*)(base + rr * pitch + 4 * cb),
                                                     4, 0, 0);
                }
            }
        }
    };
    // species -> F * species in place (F * species <= 24: no byte overflows
    // into the next)
    auto scale = [&](int slot) {
        uint8_t* base = win + slot * plane_bytes;
        for (int i = threadIdx.x; i < nitems; i += kSlabBlock) {
            const int rr = i / nd, j = i - rr * nd;
            uint32_t* w = (uint32_t*)(base + rr * pitch + 4 * j);
            *w = F == 8 ? *w << 3 : *w * 6u;
        }
    };
    // accumulators [species][shell][word] with 16-bit fields: for F = 8, word 0
    // holds l = 0 and 2, word 1 l = 1 and 3; for F = 6, word w holds l = 2 w
    // and 2 w + 1
    uint32_t acc[KF][kMaxShells][NWD];
#pragma unroll
    for (int k = 0; k < KF; ++k)
#pragma unroll
        for (int s = 0; s < kMaxShells; ++s)
#pragma unroll
            for (int w = 0; w < NWD; ++w) acc[k][s][w] = 0;
    stage(z0, 0);
    stage(z0 + 1, 1);
    stage(z0 + 2, 2);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    scale(0);
    scale(1);
    scale(2);
    __syncthreads();
    const int ny = min(kSlabY, L1 - y0);
    const int ncells = ny * L0;
    for (int z = z0; z < z1; ++z) {
        const bool more = z + 3 < z1 + 2;  // planes up to z1 + 1 are read
        const int sl = z - z0;
        if (more) stage(z + 3, (sl + 3) & 3);  // in flight while plane z is counted
        const int pb0 = ((sl + 0) & 3) * plane_bytes, pb1 = ((sl + 1) & 3) * plane_bytes,
                  pb2 = ((sl + 2) & 3) * plane_bytes;
        int ly = threadIdx.x / L0, x = threadIdx.x - ly * L0;
        const int dly = kSlabBlock / L0, dx = kSlabBlock - dly * L0;
        for (int c = threadIdx.x; c < ncells; c += kSlabBlock) {
            const int cell = (ly + kHalo) * pitch + (x + kHalo) * m;
#pragma unroll
            for (int b = 0; b < m; ++b) {
                const int k8 = win[pb0 + cell + b];
                uint32_t e[KF];
#pragma unroll
                for (int kk = 0; kk < KF; ++kk) e[kk] = k8 == F * kk ? 1u : 0u;
#pragma unroll
                for (int s = 0; s < kMaxShells; ++s) {
                    if (s < S) {
                        uint32_t h = 0;
#pragma unroll
                        for (int n = 0; n < G.Z[s]; ++n) {
                            if (!positive(G.v[s][n])) continue;
                            const Nb nb = nb_of(G, b, G.v[s][n][0], G.v[s][n][1], G.v[s][n][2]);
                            const int pbz = nb.dz == 0 ? pb0 : (nb.dz == 1 ? pb1 : pb2);
                            h = shl1_add(win[pbz + cell + nb.dy * pitch + nb.dx * m + nb.bt], h);
                        }
                        // F-bit fields (<= 12 each) -> words of 16-bit fields
                        uint32_t wd[NWD];
                        if constexpr (F == 8) {
                            wd[0] = h & 0x00FF00FFu;
                            wd[1] = (h >> 8) & 0x00FF00FFu;
                        } else {
#pragma unroll
                            for (int w = 0; w < NWD; ++w)
                                wd[w] = ((h >> (12 * w)) & 0x3Fu) | (((h >> (12 * w + 6)) & 0x3Fu) << 16);
                        }
#pragma unroll
                        for (int kk = 0; kk < KF; ++kk)
#pragma unroll
                            for (int w = 0; w < NWD; ++w) acc[kk][s][w] = __umul24(wd[w], e[kk]) + acc[kk][s][w];
                    }
                }
                // one site's reads at a time: registers for two workgroups per CU
                __builtin_amdgcn_sched_barrier(0);
            }
            ly += dly;
            x += dx;
            if (x >= L0) {
                x -= L0;
                ++ly;
            }
        }
        if (more) {
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            scale((sl + 3) & 3);
        }
        __syncthreads();
    }
    // wave sums of H[s][k][l] into LDS (the window is free after the last
    // barrier), the workgroup's totals, then one atomic per directed count:
    // a few dozen atomics per workgroup instead of that many per wave
    constexpr int NW = kSlabBlock / 64;
    constexpr int KK = KF * KF;                  // H[k][l] entries of one shell
    uint32_t* red = (uint32_t*)win;              // [NW][kMaxShells][KK]
    uint32_t* tot = red + NW * kMaxShells * KK;  // [kMaxShells][KK]
#pragma unroll
    for (int s = 0; s < kMaxShells; ++s) {
#pragma unroll
        for (int k = 0; k < KF; ++k) {
#pragma unroll
            for (int l = 0; l < KF; ++l) {
                // field of l: F = 8 words hold (0, 2) and (1, 3); F = 6 words (2w, 2w + 1)
                const int w = F == 8 ? (l & 1) : l >> 1, hi = F == 8 ? l >> 1 : l & 1;
                const uint32_t h = wave_sum(hi ? acc[k][s][w] >> 16 : acc[k][s][w] & 0xFFFFu);
                if (lane == 0) red[(wave * kMaxShells + s) * KK + k * KF + l] = h;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < kMaxShells * KK) {
        uint32_t v = 0;
        for (int w = 0; w < NW; ++w) v += red[w * kMaxShells * KK + threadIdx.x];
        tot[threadIdx.x] = v;
    }
    __syncthreads();
    if (threadIdx.x < kMaxShells * KK) {
        const int s = threadIdx.x / KK, k = (threadIdx.x % KK) / KF, l = threadIdx.x % KF;
        if (s < S && k < K && l < K) {
            const uint32_t c = tot[s * KK + KF * k + l] + tot[s * KK + KF * l + k];
            if (c != 0)
                atomicAdd((unsigned long long*)&counts[(int64_t)blockIdx.z * S * K * K + (s * K + k) * K + l],
                          (unsigned long long)c);
        }
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Kernel resolution: (lattice, counter encoding, window preset) -> kernels.
// Stream kernels exist for the runtime geometry and every preset of the
// lattice; persistent kernels use the runtime geometry only.
// ---------------------------------------------------------------------------
int encoding_of(int K) { return K <= 4 ? 1 : (K == 5 ? 3 : 2); }
int field_bits_of(int K) { return K == 5 ? 6 : 8; }

template <int LAT, int E>
static const void* stream_kernel(int preset, int nbuf)
{
    if constexpr (E != 2) {
        if constexpr (LAT == SMCX_BCC) {
            if (preset == 0) return (const void*)k_ministep<LAT, E, GeoFix<0>, 1>;
            if (preset == 1) return (const void*)k_ministep<LAT, E, GeoFix<1>, 1>;
        } else {
            if (preset == 2) return (const void*)k_ministep<LAT, E, GeoFix<2>, 1>;
            if (preset == 3) return (const void*)k_ministep<LAT, E, GeoFix<3>, 1>;
        }
    }
    if (preset >= 0) return nullptr;
    if (nbuf == 2) return (const void*)k_ministep<LAT, E, GeoRt, 2>;
    return (const void*)k_ministep<LAT, E, GeoRt, 1>;
}

template <int LAT, int E>
static const void* persistent_kernel()
{
    return (const void*)k_persistent<LAT, E, GeoRt>;
}


// Row kernels: compile-time species / shell counts for the 4-species BCC
// and 5-species FCC alloys with 4 or 2 shells, runtime counts otherwise (at
// about half the speed: the 2-shell BCC lattice of 795^3 cells ran 2.2x
// faster with its counts fixed).
template <int LAT, int E, int MAXB>
static const void* row_kernel_e(int K, int S)
{
    if constexpr (LAT == SMCX_BCC && E == 1) {
        if (K == 4 && S == 4) return (const void*)k_rows<LAT, E, GeoRow<4, 4>, MAXB>;
        if (K == 4 && S == 2) return (const void*)k_rows<LAT, E, GeoRow<4, 2>, MAXB>;
    }
    if constexpr (LAT == SMCX_FCC && E == 3) {
        if (K == 5 && S == 4) return (const void*)k_rows<LAT, E, GeoRow<5, 4>, MAXB>;
        if (K == 5 && S == 2) return (const void*)k_rows<LAT, E, GeoRow<5, 2>, MAXB>;
    }
    return (const void*)k_rows<LAT, E, GeoRow<0, 0>, MAXB>;
}

template <int MAXB>
static const void* row_kernel_b(int lattice, int K, int S)
{
    const int e = encoding_of(K);
    if (lattice == SMCX_BCC)
        return e == 1 ? row_kernel_e<SMCX_BCC, 1, MAXB>(K, S)
                      : (e == 3 ? row_kernel_e<SMCX_BCC, 3, MAXB>(K, S) : row_kernel_e<SMCX_BCC, 2, MAXB>(K, S));
    return e == 1 ? row_kernel_e<SMCX_FCC, 1, MAXB>(K, S)
                  : (e == 3 ? row_kernel_e<SMCX_FCC, 3, MAXB>(K, S) : row_kernel_e<SMCX_FCC, 2, MAXB>(K, S));
}

// The row kernel of compile-time row preset PI or a later one.
template <int PI>
static const void* row_preset_kernel(int preset)
{
    if constexpr (PI < kNumRowPresets) {
        if (preset == PI) {
            constexpr RowPreset q = kRowPresets[PI];
            static_assert(q.K <= 4, "row presets use 8-bit fields");
            constexpr int B = (q.rt0 * q.rt1 * q.rt2 + 63) / 64 * 64;
            return (const void*)k_rows<q.lattice, 1, GeoRowFix<PI>, (B <= kBlock ? kBlock : kMaxRowBlock)>;
        }
        return row_preset_kernel<PI + 1>(preset);
    } else {
        return nullptr;
    }
}

const void* row_kernel(int lattice, int K, int S, int block, int preset)
{
    if (preset >= 0) return row_preset_kernel<0>(preset);
    return block <= kBlock ? row_kernel_b<kBlock>(lattice, K, S) : row_kernel_b<kMaxRowBlock>(lattice, K, S);
}

const void* sweep_kernel(int lattice, int K, bool persistent, int preset, int nbuf)
{
    const int e = encoding_of(K);
    if (lattice == SMCX_BCC) {
        if (persistent) return e == 1 ? persistent_kernel<SMCX_BCC, 1>() : (e == 3 ? persistent_kernel<SMCX_BCC, 3>() : persistent_kernel<SMCX_BCC, 2>());
        return e == 1 ? stream_kernel<SMCX_BCC, 1>(preset, nbuf) : (e == 3 ? stream_kernel<SMCX_BCC, 3>(preset, nbuf) : stream_kernel<SMCX_BCC, 2>(preset, nbuf));
    }
    if (persistent) return e == 1 ? persistent_kernel<SMCX_FCC, 1>() : (e == 3 ? persistent_kernel<SMCX_FCC, 3>() : persistent_kernel<SMCX_FCC, 2>());
    return e == 1 ? stream_kernel<SMCX_FCC, 1>(preset, nbuf) : (e == 3 ? stream_kernel<SMCX_FCC, 3>(preset, nbuf) : stream_kernel<SMCX_FCC, 2>(preset, nbuf));
}

hipError_t launch_sweep(const void* kernel, dim3 grid, int block, size_t lds, hipStream_t st, const SweepArgs& a)
{
    if (!kernel) return hipErrorInvalidDeviceFunction;
    SweepArgs copy = a;
    void* args[] = {&copy};
    return hipLaunchKernel(kernel, grid, dim3(block), args, lds, st);
}

hipError_t set_sweep_lds_limit(const void* kernel, size_t lds)
{
    return hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t sweep_occupancy(const void* kernel, int block, size_t lds, int* blocks_per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, kernel, block, lds);
}

hipError_t launch_pack(int lattice, int K, bool unpack, bool planar, uint8_t* occ, uint8_t* ws,
                       const RepDev* reps, int r, int64_t nrows, int nrep, hipStream_t st)
{
    // a workgroup per row (padded rows to pack, natural rows to unpack) of
    // replica r, or with r < 0 a grid row per replica (nrep of them, nrows
    // the largest replica's rows), up to 8 rows per workgroup
    int64_t nb = r < 0 ? (nrows + 7) / 8 : nrows;
    if (nb > 65536) nb = 65536;
    if (nb < 1) nb = 1;
    if (r < 0 && (nrep < 1 || nrep > 65535)) return hipErrorInvalidValue;
    const dim3 g((unsigned)nb, r < 0 ? (unsigned)nrep : 1u), b(kBlock);
    const int F = field_bits_of(K);
    auto go = [&](auto mt, auto pt) {
        constexpr int M = decltype(mt)::value;
        constexpr bool PL = decltype(pt)::value;
        if (unpack) hipLaunchKernelGGL((k_unpack<M, PL>), g, b, 0, st, occ, ws, reps, r, F);
        else hipLaunchKernelGGL((k_pack<M, PL>), g, b, 0, st, occ, ws, reps, r, F);
    };
    using T2 = std::integral_constant<int, 2>;
    using T4 = std::integral_constant<int, 4>;
    using Y = std::true_type;
    using N = std::false_type;
    if (lattice == SMCX_BCC) {
        if (planar) go(T2{}, Y{}); else go(T2{}, N{});
    } else {
        if (planar) go(T4{}, Y{}); else go(T4{}, N{});
    }
    return hipGetLastError();
}

hipError_t launch_validate(const uint8_t* occ, int64_t n, int K, int32_t* bad, hipStream_t st)
{
    int64_t nb = (n + kBlock - 1) / kBlock;
    if (nb > 65536) nb = 65536;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_validate, dim3((unsigned)nb), dim3(kBlock), 0, st, occ, n, K, bad);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Replica exchange.  k_energy: E_r = 1/2 sum_{s,k,l} C_r[s][k][l] V[s][k][l],
// accumulated s, k, l ascending in binary64, one thread per replica (the
// order fixes the rounding, the same as the host-side energy).  k_exchange:
// one round of trades between neighbouring temperature slots (i, i + 1),
// i = round mod 2, round mod 2 + 2, ...: with a = rep_at[i], b = rep_at[i+1]
// and x = (beta_slot[i] - beta_slot[i+1]) (E_a - E_b), the trade is taken
// when x >= 0, else when u < exp(x) (u from Philox on counter
// (i, 0, round, 0xffffffff), which no trial uses); near-ties
// (|u - exp(x)| < 1e-12) go to the tie log as {-1, round, i, decision}.
// One workgroup: every pair of the round has its own thread, so the pairs'
// slots, stats and trades never collide.  Then every replica's new beta is
// written to each of the n_rows rows the next sweeps read.  rep_at entries
// outside [0, R) leave their pair (and their replica's beta) untouched.
// ---------------------------------------------------------------------------
__global__ void k_energy(const int64_t* C, const double* V, int R, int SKK, double* E)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const int64_t* c = C + (int64_t)r * SKK;
    double acc = 0.0;
    for (int i = 0; i < SKK; ++i) acc = acc + (double)c[i] * V[i];
    E[r] = 0.5 * acc;
}

__global__ __launch_bounds__(kBlock) void k_exchange(const double* E, const double* beta_slot, int32_t* rep_at, int R,
                                                     uint64_t seed, uint32_t round, double* beta_rows, int n_rows,
                                                     int64_t* xstats, smcx_tie* ties, int32_t tie_cap,
                                                     int32_t* tie_count)
{
    for (int i = (int)(round & 1u) + 2 * (int)threadIdx.x; i + 1 < R; i += 2 * (int)blockDim.x) {
        const int a = rep_at[i], b = rep_at[i + 1];
        if (a < 0 || a >= R || b < 0 || b >= R) continue;
        const double x = (beta_slot[i] - beta_slot[i + 1]) * (E[a] - E[b]);
        bool acc = true, tie = false;
        if (!(x >= 0.0)) {
            uint32_t w0, w1, w2, w3;
            philox4x32_10((uint32_t)i, 0u, round, 0xffffffffu, (uint32_t)seed, (uint32_t)(seed >> 32), w0, w1, w2,
                          w3);
            (void)w0;
            (void)w3;
            const double P = exp(x);
            const double u = (double)(((uint64_t)w1 << 21) | (uint64_t)(w2 >> 11)) * 0x1p-53;
            acc = u < P;
            tie = fabs(u - P) < 1e-12;
        }
        if (tie) {
            const int slot = atomicAdd(tie_count, 1);
            if (slot < tie_cap) {
                smcx_tie e;
                e.replica = -1;
                e.sweep = round;
                e.site = i;
                e.decision = acc ? 1 : 0;
                e.pad = 0;
                ties[slot] = e;
            }
        }
        xstats[2 * i] += 1;
        if (acc) {
            xstats[2 * i + 1] += 1;
            rep_at[i] = b;
            rep_at[i + 1] = a;
        }
    }
    __syncthreads();  // every trade of the round is in rep_at
    for (int j = threadIdx.x; j < R; j += blockDim.x) {
        const int r = rep_at[j];
        if (r < 0 || r >= R) continue;
        const double bj = beta_slot[j];
        for (int row = 0; row < n_rows; ++row) beta_rows[(int64_t)row * R + r] = bj;
    }
}

// Heat capacity per site (units of k_B) of every (step, replica) from its
// recorded energies E[s][j][r], j < n_rec: c = (beta beta) v / N with
// m = (sum_j E) / n_rec and v = (sum_j (E - m)^2) / n_rec, j ascending in
// binary64 (the canonical fluctuation formula); beta = beta_steps[s][r].
__global__ void k_heat_capacity(const double* E, const double* beta_steps, const RepDev* reps, int n_steps,
                                int n_rec, int R, double* cv)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_steps * R) return;
    const int64_t s = i / R;
    const int r = (int)(i - s * R);
    const double* e = E + s * n_rec * R + r;
    double m = 0.0;
    for (int j = 0; j < n_rec; ++j) m = m + e[(int64_t)j * R];
    m = m / (double)n_rec;
    double v = 0.0;
    for (int j = 0; j < n_rec; ++j) {
        const double d = e[(int64_t)j * R] - m;
        v = v + d * d;
    }
    v = v / (double)n_rec;
    const double b = beta_steps[i];
    cv[i] = b * b * v / (double)reps[r].N;
}

hipError_t launch_heat_capacity(const double* E, const double* beta_steps, const RepDev* reps, int n_steps, int n_rec,
                                int R, double* cv, hipStream_t st)
{
    const int64_t n = (int64_t)n_steps * R;
    hipLaunchKernelGGL(k_heat_capacity, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, E, beta_steps,
                       reps, n_steps, n_rec, R, cv);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Local energies and clusters of low-energy sites.
//
// k_local_energy: e_i = 1/2 sum_s sum_t n_i[s][t] V_s[sigma_i][t] (s, t
// ascending, binary64), n_i[s][t] counted from the natural layout with the
// periodic wrap.  A thread takes a conventional cell and each of its basis
// sites in turn, so every neighbour displacement is a compile-time constant.
//
// Clusters: site i is marked when e_i <= threshold; marked nearest neighbours
// join.  parent[] starts as i (marked) or -1, and always points at a smaller
// or equal index: a union hooks the larger of two roots under the smaller
// (compare-and-swap), a find halves the path to an ancestor.  The smallest
// site of a cluster is therefore its final root, whatever the order of the
// unions.  Every access to parent[] is an agent-scope atomic (the L2 of one
// XCD does not see another's plain stores); a failed hook continues from the
// value the swap returned, and a find only descends, so both loops end.
// ---------------------------------------------------------------------------
template <int LAT, int B>
__device__ __forceinline__ double local_energy_at(const uint8_t* occ, int x, int y, int z, int L0, int L1, int L2,
                                                  int K, int S, const double* Vs)
{
    constexpr Geometry G = kGeom[LAT];
    constexpr int m = G.m;
    uint64_t acc[kMaxShells];
#pragma unroll
    for (int s = 0; s < kMaxShells; ++s) {
        uint64_t a = 0;
        if (s < S) {
#pragma unroll
            for (int n = 0; n < G.Z[s]; ++n) {
                const Nb nb = nb_of(G, B, G.v[s][n][0], G.v[s][n][1], G.v[s][n][2]);
                int xx = x + nb.dx, yy = y + nb.dy, zz = z + nb.dz;
                xx += xx < 0 ? L0 : (xx >= L0 ? -L0 : 0);
                yy += yy < 0 ? L1 : (yy >= L1 ? -L1 : 0);
                zz += zz < 0 ? L2 : (zz >= L2 ? -L2 : 0);
                const uint32_t t = occ[nb.bt + m * (xx + L0 * (yy + L1 * zz))] & 7u;  // species < K <= 8
                a += (uint64_t)1 << (8 * t);
            }
        }
        acc[s] = a;
    }
    const int p = min((int)occ[B + m * (x + L0 * (y + L1 * z))], K - 1);  // checked < K at init
    double e = 0.0;
#pragma unroll
    for (int s = 0; s < kMaxShells; ++s)
        if (s < S)
            for (int t = 0; t < K; ++t)
                e = e + (double)(int)((acc[s] >> (8 * t)) & 0xff) * Vs[(s * K + p) * K + t];
    return 0.5 * e;
}

template <int LAT, int B>
__device__ __forceinline__ void local_energy_sites(const uint8_t* occ, int c, int L0, int L1, int L2, int K, int S,
                                                   const double* Vs, double* e)
{
    constexpr int m = kGeom[LAT].m;
    if constexpr (B < m) {
        const int x = c % L0, cr = c / L0, y = cr % L1, z = cr / L1;
        e[B + m * c] = local_energy_at<LAT, B>(occ, x, y, z, L0, L1, L2, K, S, Vs);
        local_energy_sites<LAT, B + 1>(occ, c, L0, L1, L2, K, S, Vs, e);
    }
}

template <int LAT>
__global__ __launch_bounds__(kBlock) void k_local_energy(const uint8_t* occ, int L0, int L1, int L2, int K, int S,
                                                         const double* V, double* e)
{
    __shared__ double Vs[kMaxShells * kMaxK * kMaxK];
    for (int i = threadIdx.x; i < S * K * K; i += blockDim.x) Vs[i] = V[i];
    __syncthreads();
    const int ncell = L0 * L1 * L2;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ncell; c += gridDim.x * blockDim.x)
        local_energy_sites<LAT, 0>(occ, c, L0, L1, L2, K, S, Vs, e);
}

// Local energies for K <= 4 from LDS tiles, the layout of
// k_pair_counts_tiled: TX x (256 / TX) lanes over x and y, 16 sites deep in
// z, the tile plus a 2-cell halo staged once; a shell's neighbours are
// counted into 8-bit fields of one word (offsets fixed at compile time) and
// e is formed in the order of k_local_energy (s, then t).
template <int LAT, int TX>
__global__ __launch_bounds__(kBlock) void k_local_energy_tiled(const uint8_t* occ, int L0, int L1, int L2, int K,
                                                               int S, const double* V, double* e)
{
    constexpr Geometry G = kGeom[LAT];
    constexpr int m = G.m;
    constexpr int TY = kBlock / TX, TZ = 16;
    constexpr int WX = TX + 2 * kHalo, WY = TY + 2 * kHalo, WZ = TZ + 2 * kHalo;
    constexpr int LP = WX * m, PL = LP * WY;
    __shared__ __align__(16) uint8_t win[PL * WZ];
    __shared__ double Vs[kMaxShells * 4 * 4];
    for (int i = threadIdx.x; i < S * K * K; i += blockDim.x) Vs[i] = V[i];
    const int ntx = (L0 + TX - 1) / TX, nty = (L1 + TY - 1) / TY, ntz = (L2 + TZ - 1) / TZ;
    const int64_t ntiles = (int64_t)ntx * nty * ntz;
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    auto wrap = [](int v, int L) {
        v += v < 0 ? L : 0;
        v -= v >= L ? L : 0;
        return v >= L ? v % L : v;  // only lattices narrower than a tile wrap twice
    };
    for (int64_t ti = blockIdx.x; ti < ntiles; ti += gridDim.x) {
        const int tx = (int)(ti % ntx);
        const int64_t tr = ti / ntx;
        const int ty = (int)(tr % nty), tz = (int)(tr / nty);
        const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
        __syncthreads();  // every lane is done with the previous tile (and Vs is in place)
        for (int c = threadIdx.x; c < WX * WY * WZ; c += blockDim.x) {
            const int wx = c % WX, wr = c / WX, wy = wr % WY, wz = wr / WY;
            const int x = wrap(x0 + wx - kHalo, L0), y = wrap(y0 + wy - kHalo, L1), z = wrap(z0 + wz - kHalo, L2);
            const int64_t cell = x + (int64_t)L0 * (y + (int64_t)L1 * z);
            uint8_t* d = win + (wz * WY + wy) * LP + wx * m;
            if constexpr (m == 2) *(uint16_t*)d = *(const uint16_t*)(occ + 2 * cell);
            else *(uint32_t*)d = *(const uint32_t*)(occ + 4 * cell);
        }
        __syncthreads();
        if (x0 + lx >= L0 || y0 + ly >= L1) continue;
        for (int lz = 0; lz < TZ && z0 + lz < L2; ++lz) {
            const int64_t cell = (x0 + lx) + (int64_t)L0 * ((y0 + ly) + (int64_t)L1 * (z0 + lz));
#pragma unroll
            for (int b = 0; b < m; ++b) {
                const int base = ((lz + kHalo) * WY + (ly + kHalo)) * LP + (lx + kHalo) * m + b;
                const int p = min((int)win[base], K - 1);  // checked < K at init
                uint32_t h[kMaxShells];
#pragma unroll
                for (int s = 0; s < kMaxShells; ++s) {
                    uint32_t a = 0;
                    if (s < S) {
                        uint32_t v[kMaxZ];
#pragma unroll
                        for (int n = 0; n < G.Z[s]; ++n) {
                            const Nb nb = nb_of(G, b, G.v[s][n][0], G.v[s][n][1], G.v[s][n][2]);
                            v[n] = win[base + nb.dz * PL + nb.dy * LP + m * nb.dx + (nb.bt - b)];
                        }
#pragma unroll
                        for (int n = 0; n < G.Z[s]; ++n) a += 1u << (8 * (v[n] & 3u));
                    }
                    h[s] = a;
                }
                double en = 0.0;
#pragma unroll
                for (int s = 0; s < kMaxShells; ++s)
                    if (s < S)
                        for (int t = 0; t < K; ++t)
                            en = en + (double)(int)((h[s] >> (8 * t)) & 0xff) * Vs[(s * K + p) * K + t];
                e[b + m * cell] = 0.5 * en;
            }
        }
    }
}

__device__ __forceinline__ int32_t par_load(const int32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void par_store(int32_t* p, int32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x.  HALVE: point x at its grandparent on the way (while trees
// still merge any ancestor will do); without it the walk only reads: in the
// final labelling a halving store could race with a store of the root and
// leave an older ancestor as a label, so there the path is pointed at the
// root instead, which every writer agrees on.
// (The final labelling reads with plain loads: the trees no longer change,
// and an out-of-date entry is still an ancestor.)
template <bool HALVE>
__device__ __forceinline__ int32_t cluster_find(int32_t* parent, int32_t x)
{
    while (true) {
        const int32_t p = HALVE ? par_load(parent + x) : parent[x];
        if (p == x) return x;
        const int32_t gp = HALVE ? par_load(parent + p) : parent[p];
        if (HALVE && gp != p) par_store(parent + x, gp);  // gp is an ancestor of x
        x = gp;
    }
}

__global__ void k_cluster_init(const double* e, int N, double threshold, int32_t* parent, int32_t* size)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
        parent[i] = e[i] <= threshold ? i : -1;
        size[i] = 0;
    }
}

template <int LAT, int B>
__device__ __forceinline__ void cluster_hook_site(int32_t* parent, int c, int L0, int L1, int L2)
{
    constexpr Geometry G = kGeom[LAT];
    constexpr int m = G.m;
    if constexpr (B < m) {
        const int i = B + m * c;
        if (parent[i] >= 0) {  // marks never change during the unions: a plain load will do
            const int x = c % L0, cr = c / L0, y = cr % L1, z = cr / L1;
#pragma unroll
            for (int n = 0; n < G.Z[0]; ++n) {
                const Nb nb = nb_of(G, B, G.v[0][n][0], G.v[0][n][1], G.v[0][n][2]);
                int xx = x + nb.dx, yy = y + nb.dy, zz = z + nb.dz;
                xx += xx < 0 ? L0 : (xx >= L0 ? -L0 : 0);
                yy += yy < 0 ? L1 : (yy >= L1 ? -L1 : 0);
                zz += zz < 0 ? L2 : (zz >= L2 ? -L2 : 0);
                const int j = nb.bt + m * (xx + L0 * (yy + L1 * zz));
                if (j <= i || parent[j] < 0) continue;  // each marked pair once
                int a = i, b = j;
                while (true) {
                    a = cluster_find<true>(parent, a);
                    b = cluster_find<true>(parent, b);
                    if (a == b) break;
                    if (a < b) {
                        const int t = a;
                        a = b;
                        b = t;
                    }
                    int expected = a;  // hook root a under the smaller root b
                    if (__hip_atomic_compare_exchange_strong(parent + a, &expected, b, __ATOMIC_RELAXED,
                                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                        break;
                    a = expected;  // a was no longer a root: go on from its parent (< a)
                }
            }
        }
        cluster_hook_site<LAT, B + 1>(parent, c, L0, L1, L2);
    }
}

template <int LAT>
__global__ void k_cluster_hook(int32_t* parent, int L0, int L1, int L2)
{
    const int ncell = L0 * L1 * L2;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ncell; c += gridDim.x * blockDim.x)
        cluster_hook_site<LAT, 0>(parent, c, L0, L1, L2);
}

__global__ void k_cluster_flatten(int32_t* parent, int N, int32_t* size, int64_t* n_clusters)
{
    int roots = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
        if (parent[i] < 0) continue;
        // the trees are final, each with one root: point the whole path at
        // the root (every thread that writes an entry writes that same root)
        const int32_t r = cluster_find<false>(parent, i);
        for (int32_t x = i; x != r;) {
            const int32_t next = parent[x];
            parent[x] = r;
            x = next;
        }
        atomicAdd(size + r, 1);
        roots += r == i;
    }
    const int w = wave_sum_i(roots);
    if ((threadIdx.x & 63) == 0 && w) atomicAdd((unsigned long long*)n_clusters, (unsigned long long)w);
}

hipError_t launch_local_energy(int lattice, const uint8_t* occ, const int32_t* L, int K, int S, const double* V,
                               double* e, hipStream_t st)
{
    const int64_t ncell = (int64_t)L[0] * L[1] * L[2];
    if (K <= 4) {
        const bool wide = L[0] >= 48;
        const int TX = wide ? 64 : 16, TY = kBlock / TX;
        const int64_t ntiles = (int64_t)((L[0] + TX - 1) / TX) * ((L[1] + TY - 1) / TY) * ((L[2] + 15) / 16);
        const unsigned g = (unsigned)std::min<int64_t>(ntiles, 1 << 20);
        auto go = [&](auto kern) { hipLaunchKernelGGL(kern, dim3(g), dim3(kBlock), 0, st, occ, L[0], L[1], L[2], K, S, V, e); };
        if (lattice == SMCX_BCC) {
            if (wide) go(k_local_energy_tiled<SMCX_BCC, 64>); else go(k_local_energy_tiled<SMCX_BCC, 16>);
        } else {
            if (wide) go(k_local_energy_tiled<SMCX_FCC, 64>); else go(k_local_energy_tiled<SMCX_FCC, 16>);
        }
        return hipGetLastError();
    }
    const unsigned nb = (unsigned)std::min<int64_t>(std::max<int64_t>(1, (ncell + kBlock - 1) / kBlock), 1 << 20);
    if (lattice == SMCX_BCC)
        hipLaunchKernelGGL(k_local_energy<SMCX_BCC>, dim3(nb), dim3(kBlock), 0, st, occ, L[0], L[1], L[2], K, S, V, e);
    else
        hipLaunchKernelGGL(k_local_energy<SMCX_FCC>, dim3(nb), dim3(kBlock), 0, st, occ, L[0], L[1], L[2], K, S, V, e);
    return hipGetLastError();
}

hipError_t launch_clusters(int lattice, const double* e, const int32_t* L, double threshold, int32_t* label,
                           int32_t* size, int64_t* n_clusters, hipStream_t st)
{
    const int m = lattice == SMCX_BCC ? 2 : 4;
    const int64_t ncell = (int64_t)L[0] * L[1] * L[2];
    const int N = (int)(m * ncell);
    const unsigned nbs = (unsigned)std::min<int64_t>(std::max<int64_t>(1, ((int64_t)N + kBlock - 1) / kBlock), 1 << 20);
    const unsigned nbc = (unsigned)std::min<int64_t>(std::max<int64_t>(1, (ncell + kBlock - 1) / kBlock), 1 << 20);
    hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(kBlock), 0, st, n_clusters, (int64_t)1, (int64_t)0);
    hipLaunchKernelGGL(k_cluster_init, dim3(nbs), dim3(kBlock), 0, st, e, N, threshold, label, size);
    if (lattice == SMCX_BCC)
        hipLaunchKernelGGL(k_cluster_hook<SMCX_BCC>, dim3(nbc), dim3(kBlock), 0, st, label, L[0], L[1], L[2]);
    else
        hipLaunchKernelGGL(k_cluster_hook<SMCX_FCC>, dim3(nbc), dim3(kBlock), 0, st, label, L[0], L[1], L[2]);
    // a grid-stride grid of 4096 workgroups: one count atomic per wave, not per 256 sites
    hipLaunchKernelGGL(k_cluster_flatten, dim3(std::min(nbs, 4096u)), dim3(kBlock), 0, st, label, N, size, n_clusters);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// qSRO model: trials whose energy change needs every local energy of the
// swap's interaction zone.  E_i = sum_m sum_t V_m[p][t] (n_i[m][t] / Z_m)
// + sum_m W_m[p] (n_i[m][p] / Z_m)^2 (p = sigma_i; m, then t, ascending,
// binary64).  A wave takes one trial (the same Philox draw, partner and
// acceptance rule as the pair model); its lanes take the sites of the
// affected set (a, the partner and every shell neighbour of either, in the
// host table's order), recount each one's neighbours before and after the
// swap (the swap applied to the two sites on the fly) and leave
// E_after - E_before in LDS; lane 0 adds the terms in table order, decides
// and writes the swap.  The sites are read from the natural layout; the
// partition keeps every read of a mini-step's trial clear of the other
// trials' writes (interaction-zone rule).
// ---------------------------------------------------------------------------

__device__ __forceinline__ int qsro_site_of(const QsroArgs& A, int x, int y, int z, int32_t d, int m)
{
    // d packs (dx + 8) | (dy + 8) << 8 | (dz + 8) << 16 | basis << 24
    int xx = x + (d & 0xff) - 8, yy = y + ((d >> 8) & 0xff) - 8, zz = z + ((d >> 16) & 0xff) - 8;
    xx += xx < 0 ? A.L0 : (xx >= A.L0 ? -A.L0 : 0);
    yy += yy < 0 ? A.L1 : (yy >= A.L1 ? -A.L1 : 0);
    zz += zz < 0 ? A.L2 : (zz >= A.L2 ? -A.L2 : 0);
    return (d >> 24) + m * (xx + A.L0 * (yy + A.L1 * zz));
}

// Tables of a qSRO launch in LDS: V and W, and every fraction n / Z_s
// (n = 0 .. Z_s), each the correctly rounded quotient, so a lookup gives the
// value the division would.
constexpr int kQsroFrac = kMaxZ + 1;
struct QsroTables {
    double V[kMaxShells * 8 * 8];
    double W[kMaxShells * 8];
    double F[kMaxShells * kQsroFrac];
};

__device__ __forceinline__ void qsro_tables(const QsroArgs& A, QsroTables& T)
{
    for (int i = threadIdx.x; i < A.S * A.K * A.K; i += blockDim.x) T.V[i] = A.V[i];
    for (int i = threadIdx.x; i < A.S * A.K; i += blockDim.x) T.W[i] = A.W[i];
    for (int i = threadIdx.x; i < A.S * kQsroFrac; i += blockDim.x) {
        const int s = i / kQsroFrac, n = i - s * kQsroFrac;
        T.F[i] = (double)n / (double)A.Z[s];
    }
    __syncthreads();
}

__device__ __forceinline__ double qsro_energy(const QsroArgs& A, const QsroTables& T, int p,
                                              const uint64_t (&n)[kMaxShells])
{
    double acc = 0.0;
    for (int s = 0; s < A.S; ++s)
        for (int t = 0; t < A.K; ++t)
            acc = acc + T.V[(s * A.K + p) * A.K + t] * T.F[s * kQsroFrac + (int)((n[s] >> (8 * t)) & 0xff)];
    for (int s = 0; s < A.S; ++s) {
        const double f = T.F[s * kQsroFrac + (int)((n[s] >> (8 * p)) & 0xff)];
        acc = acc + T.W[s * A.K + p] * (f * f);
    }
    return acc;
}

template <int LAT>
__global__ __launch_bounds__(64) void k_qsro_ministep(QsroArgs A)
{
    constexpr int m = kGeom[LAT].m;
    __shared__ double term[kQsroMaxAff];
    __shared__ QsroTables tab;
    qsro_tables(A, tab);
    const int lane = threadIdx.x;
    const int ncell = A.ncx * A.ncy * A.ncz;
    const int32_t* ox = A.org;
    const int32_t* oy = ox + A.ncx + 1;
    const int32_t* oz = oy + A.ncy + 1;
    int att = 0, nacc = 0, ntie = 0;
    for (int c = blockIdx.x; c < ncell; c += gridDim.x) {
        const int cx = c % A.ncx, cy = (c / A.ncx) % A.ncy, cz = c / (A.ncx * A.ncy);
        if (A.o0 >= ox[cx + 1] - ox[cx] || A.o1 >= oy[cy + 1] - oy[cy] || A.o2 >= oz[cz + 1] - oz[cz]) continue;
        const int x = ox[cx] + A.o0, y = oy[cy] + A.o1, z = oz[cz] + A.o2;
        const int a = A.b + m * (x + A.L0 * (y + A.L1 * z));
        uint32_t w0, w1, w2, w3;
        philox4x32_10((uint32_t)a, 0u, A.sweep, A.replica, (uint32_t)A.seed, (uint32_t)(A.seed >> 32), w0, w1, w2, w3);
        (void)w3;
        const int k = (int)__umulhi(w0, (uint32_t)A.Z1);
        const int bsite = qsro_site_of(A, x, y, z, A.nbr[A.b * A.sumZ + k], m);
        const int p = A.occ[a], q = A.occ[bsite];
        ++att;
        if (p == q) continue;
        const int32_t* list = A.aff + (int64_t)(A.b * A.Z1 + k) * (1 + A.naff_max);
        const int naff = list[0];
        for (int i = lane; i < naff; i += 64) {
            const int j = qsro_site_of(A, x, y, z, list[1 + i], m);
            const int jb = j % m, jc = j / m;
            const int jx = jc % A.L0, jy = (jc / A.L0) % A.L1, jz = jc / (A.L0 * A.L1);
            const int sj = A.occ[j];
            const int sj2 = j == a ? q : (j == bsite ? p : sj);
            uint64_t nb[kMaxShells], na[kMaxShells];
            const int32_t* nl = A.nbr + jb * A.sumZ;
            int off = 0;
            for (int s = 0; s < kMaxShells; ++s) {
                uint64_t cb = 0, ca = 0;
                if (s < A.S) {
                    for (int n = 0; n < A.Z[s]; ++n) {
                        const int xs = qsro_site_of(A, jx, jy, jz, nl[off + n], m);
                        const int v = A.occ[xs];
                        const int v2 = xs == a ? q : (xs == bsite ? p : v);
                        cb += (uint64_t)1 << (8 * (v & 7));
                        ca += (uint64_t)1 << (8 * (v2 & 7));
                    }
                    off += A.Z[s];
                }
                nb[s] = cb;
                na[s] = ca;
            }
            term[i] = qsro_energy(A, tab, min(sj2, A.K - 1), na) - qsro_energy(A, tab, min(sj, A.K - 1), nb);
        }
        __syncthreads();
        if (lane == 0) {
            double dE = 0.0;
            for (int i = 0; i < naff; ++i) dE = dE + term[i];
            bool acc = true, tie = false;
            if (!(dE <= 0.0)) {
                const double P = exp(-(A.beta * dE));
                const double u = (double)(((uint64_t)w1 << 21) | (uint64_t)(w2 >> 11)) * 0x1p-53;
                acc = u < P;
                tie = fabs(u - P) < 1e-12;
            }
            if (tie) {
                ++ntie;
                const int slot = atomicAdd(A.tie_count, 1);
                if (slot < A.tie_cap) {
                    smcx_tie e;
                    e.replica = (int32_t)A.replica;
                    e.sweep = A.sweep;
                    e.site = a;
                    e.decision = acc ? 1 : 0;
                    e.pad = 0;
                    A.ties[slot] = e;
                }
            }
            if (acc) {
                ++nacc;
                A.occ[a] = (uint8_t)q;
                A.occ[bsite] = (uint8_t)p;
            }
        }
        __syncthreads();  // the terms are free again
    }
    if (lane == 0) {
        // this workgroup's own counter slot (no other workgroup of the
        // launch writes it; launches on one stream follow each other), so no
        // atomics: thousands of atomics on one address would serialise
        int64_t* slot = A.slots + 3 * (int64_t)blockIdx.x;
        slot[0] += att;
        slot[1] += nacc;
        slot[2] += ntie;
    }
}

// The same trial with its neighbourhood staged: the wave first copies the box
// of (2 reach + 1)^3 cells around the active site's cell (periodic, one load
// per cell of m bytes) into LDS, then every read of the affected sites and
// their neighbours is an LDS byte at a fixed offset from the site's own (no
// wrap arithmetic, no scattered L2 loads).  Each lattice site appears once in
// the box because every edge is at least 2 reach + 1 cells; sites of the box
// that the trial does not read may be written by other trials of the
// mini-step meanwhile, which is harmless.  Terms, order of the sum, decision
// and the near-tie log are those of k_qsro_ministep.
template <int LAT>
__global__ __launch_bounds__(64) void k_qsro_win(QsroArgs A)
{
    constexpr int m = kGeom[LAT].m;
    constexpr int WMAX = 2 * kQsroMaxReach + 1;
    using Cell = typename std::conditional<m == 4, uint32_t, uint16_t>::type;
    __shared__ double term[kQsroMaxAff];
    __shared__ QsroTables tab;
    __shared__ __align__(16) uint8_t win[WMAX * WMAX * WMAX * m];
    __shared__ int16_t nof[4 * kMaxShells * kMaxZ];  // [basis][neighbour]: window byte offset from the site
    qsro_tables(A, tab);
    const int lane = threadIdx.x;
    const int Rch = A.reach, W = 2 * Rch + 1, W3 = W * W * W;
    for (int i = lane; i < m * A.sumZ; i += 64) {
        const int b = i / A.sumZ;
        const int32_t d = A.nbr[i];
        const int dx = (d & 0xff) - 8, dy = ((d >> 8) & 0xff) - 8, dz = ((d >> 16) & 0xff) - 8;
        nof[i] = (int16_t)(((dz * W + dy) * W + dx) * m + (d >> 24) - b);
    }
    __syncthreads();
    const int ncell = A.ncx * A.ncy * A.ncz;
    const int32_t* ox = A.org;
    const int32_t* oy = ox + A.ncx + 1;
    const int32_t* oz = oy + A.ncy + 1;
    const int center = ((Rch * W + Rch) * W + Rch) * m;  // byte of basis site 0 of the active site's cell
    int att = 0, nacc = 0, ntie = 0;
    for (int c = blockIdx.x; c < ncell; c += gridDim.x) {
        const int cx = c % A.ncx, cy = (c / A.ncx) % A.ncy, cz = c / (A.ncx * A.ncy);
        if (A.o0 >= ox[cx + 1] - ox[cx] || A.o1 >= oy[cy + 1] - oy[cy] || A.o2 >= oz[cz + 1] - oz[cz]) continue;
        const int x = ox[cx] + A.o0, y = oy[cy] + A.o1, z = oz[cz] + A.o2;
        const int a = A.b + m * (x + A.L0 * (y + A.L1 * z));
        uint32_t w0, w1, w2, w3;
        philox4x32_10((uint32_t)a, 0u, A.sweep, A.replica, (uint32_t)A.seed, (uint32_t)(A.seed >> 32), w0, w1, w2, w3);
        (void)w3;
        const int k = (int)__umulhi(w0, (uint32_t)A.Z1);
        const int bsite = qsro_site_of(A, x, y, z, A.nbr[A.b * A.sumZ + k], m);
        // the box: cell (x, y, z) + (wx, wy, wz) - reach, one wrap per axis
        // (edges >= W); its loads go out with those of the two sites, whose
        // species may still show the trial to be void (p == q)
        const int p = A.occ[a], q = A.occ[bsite];
        for (int i = lane; i < W3; i += 64) {
            const int wx = i % W, wy = (i / W) % W, wz = i / (W * W);
            int xx = x + wx - Rch, yy = y + wy - Rch, zz = z + wz - Rch;
            xx += xx < 0 ? A.L0 : (xx >= A.L0 ? -A.L0 : 0);
            yy += yy < 0 ? A.L1 : (yy >= A.L1 ? -A.L1 : 0);
            zz += zz < 0 ? A.L2 : (zz >= A.L2 ? -A.L2 : 0);
            *(Cell*)(win + m * i) = *(const Cell*)(A.occ + m * (xx + A.L0 * (yy + A.L1 * zz)));
        }
        ++att;
        __syncthreads();
        if (p == q) continue;
        const int abyte = center + A.b;
        const int bbyte = abyte + nof[A.b * A.sumZ + k];
        const int32_t* list = A.aff + (int64_t)(A.b * A.Z1 + k) * (1 + A.naff_max);
        const int naff = list[0];
        for (int i = lane; i < naff; i += 64) {
            const int32_t d = list[1 + i];
            const int jb = d >> 24;
            const int jbyte = center + ((((d >> 16) & 0xff) - 8) * W + (((d >> 8) & 0xff) - 8)) * W * m +
                              ((d & 0xff) - 8) * m + jb;
            const int sj = win[jbyte];
            const int sj2 = jbyte == abyte ? q : (jbyte == bbyte ? p : sj);
            uint64_t nb[kMaxShells], na[kMaxShells];
            const int16_t* nl = nof + jb * A.sumZ;
            int off = 0;
            for (int s = 0; s < kMaxShells; ++s) {
                uint64_t cb = 0, ca = 0;
                if (s < A.S) {
                    for (int n = 0; n < A.Z[s]; ++n) {
                        const int xb = jbyte + nl[off + n];
                        const int v = win[xb];
                        const int v2 = xb == abyte ? q : (xb == bbyte ? p : v);
                        cb += (uint64_t)1 << (8 * (v & 7));
                        ca += (uint64_t)1 << (8 * (v2 & 7));
                    }
                    off += A.Z[s];
                }
                nb[s] = cb;
                na[s] = ca;
            }
            term[i] = qsro_energy(A, tab, min(sj2, A.K - 1), na) - qsro_energy(A, tab, min(sj, A.K - 1), nb);
        }
        __syncthreads();
        if (lane == 0) {
            double dE = 0.0;
            for (int i = 0; i < naff; ++i) dE = dE + term[i];
            bool acc = true, tie = false;
            if (!(dE <= 0.0)) {
                const double P = exp(-(A.beta * dE));
                const double u = (double)(((uint64_t)w1 << 21) | (uint64_t)(w2 >> 11)) * 0x1p-53;
                acc = u < P;
                tie = fabs(u - P) < 1e-12;
            }
            if (tie) {
                ++ntie;
                const int slot = atomicAdd(A.tie_count, 1);
                if (slot < A.tie_cap) {
                    smcx_tie e;
                    e.replica = (int32_t)A.replica;
                    e.sweep = A.sweep;
                    e.site = a;
                    e.decision = acc ? 1 : 0;
                    e.pad = 0;
                    A.ties[slot] = e;
                }
            }
            if (acc) {
                ++nacc;
                A.occ[a] = (uint8_t)q;
                A.occ[bsite] = (uint8_t)p;
            }
        }
        __syncthreads();  // the terms and the box are free again
    }
    if (lane == 0) {
        int64_t* slot = A.slots + 3 * (int64_t)blockIdx.x;
        slot[0] += att;
        slot[1] += nacc;
        slot[2] += ntie;
    }
}

// Sum the workgroups' counter slots into a replica's counters.
__global__ void k_qsro_reduce(const int64_t* slots, int n, int64_t* stats)
{
    int64_t v[3] = {0, 0, 0};
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        for (int c = 0; c < 3; ++c) v[c] += slots[3 * (int64_t)i + c];
    __shared__ int64_t red[3][kBlock];
    for (int c = 0; c < 3; ++c) red[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c)
            if (red[c][0]) atomicAdd((unsigned long long*)(stats + c), (unsigned long long)red[c][0]);
}

hipError_t launch_qsro_reduce(const int64_t* slots, int n, int64_t* stats, hipStream_t st)
{
    hipLaunchKernelGGL(k_qsro_reduce, dim3(1), dim3(kBlock), 0, st, slots, n, stats);
    return hipGetLastError();
}

hipError_t launch_qsro_ministep(int lattice, const QsroArgs& A, int grid, hipStream_t st)
{
    // the windowed trial where the box fits the lattice and the kernel's LDS
    // box (reach <= kQsroMaxReach), cells are aligned, and the neighbour
    // table fits; the gather kernel otherwise
    const int m = lattice == SMCX_BCC ? 2 : 4;
    const int W = 2 * A.reach + 1;
    const bool win = A.reach >= 1 && A.reach <= kQsroMaxReach && A.L0 >= W && A.L1 >= W && A.L2 >= W &&
                     ((uintptr_t)A.occ % m) == 0 && m * A.sumZ <= 4 * kMaxShells * kMaxZ;
    if (lattice == SMCX_BCC) {
        if (win) hipLaunchKernelGGL(k_qsro_win<SMCX_BCC>, dim3((unsigned)grid), dim3(64), 0, st, A);
        else hipLaunchKernelGGL(k_qsro_ministep<SMCX_BCC>, dim3((unsigned)grid), dim3(64), 0, st, A);
    } else {
        if (win) hipLaunchKernelGGL(k_qsro_win<SMCX_FCC>, dim3((unsigned)grid), dim3(64), 0, st, A);
        else hipLaunchKernelGGL(k_qsro_ministep<SMCX_FCC>, dim3((unsigned)grid), dim3(64), 0, st, A);
    }
    return hipGetLastError();
}

hipError_t launch_energy(const int64_t* C, const double* V, int R, int SKK, double* E, hipStream_t st)
{
    hipLaunchKernelGGL(k_energy, dim3((unsigned)((R + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, C, V, R, SKK, E);
    return hipGetLastError();
}

// Gradient of sum_b g_b E_b with respect to V for E_b = 1/2 <C_b, V>:
// grad[i] = 1/2 sum_b g_b C_b[i], b ascending in binary64, one thread per
// entry i of V.
__global__ void k_energy_grad(const int64_t* C, const double* g, int B, int SKK, double* grad)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= SKK) return;
    double acc = 0.0;
    for (int b = 0; b < B; ++b) acc = acc + g[b] * (double)C[(int64_t)b * SKK + i];
    grad[i] = 0.5 * acc;
}

hipError_t launch_energy_grad(const int64_t* C, const double* g, int B, int SKK, double* grad, hipStream_t st)
{
    hipLaunchKernelGGL(k_energy_grad, dim3((unsigned)((SKK + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, C, g, B,
                       SKK, grad);
    return hipGetLastError();
}

hipError_t launch_exchange(const double* E, const double* beta_slot, int32_t* rep_at, int R, uint64_t seed,
                           uint32_t round, double* beta_rows, int n_rows, int64_t* xstats, smcx_tie* ties,
                           int32_t tie_cap, int32_t* tie_count, hipStream_t st)
{
    hipLaunchKernelGGL(k_exchange, dim3(1), dim3(kBlock), 0, st, E, beta_slot, rep_at, R, seed, round, beta_rows,
                       n_rows, xstats, ties, tie_cap, tie_count);
    return hipGetLastError();
}

hipError_t launch_fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t st)
{
    int64_t nb = (n + kBlock - 1) / kBlock;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)nb), dim3(kBlock), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st)
{
    int64_t nb = (n + kBlock - 1) / kBlock;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)nb), dim3(kBlock), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_advance_counter(uint32_t* counter, uint32_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_advance_counter, dim3(1), dim3(64), 0, st, counter, n);
    return hipGetLastError();
}

hipError_t launch_pair_counts(int lattice, int K, int S, const uint8_t* occ, int64_t N, const int32_t* L,
                              int B, int64_t* counts, hipStream_t st)
{
    const int mm = lattice == SMCX_BCC ? 2 : 4;
    const int nd = (L[0] * mm) / 4 + mm;  // window dwords per row of the slab kernel
    const int slab_lds = 4 * (kSlabY + 4) * ((4 * nd + 15) & ~15);
    if (K <= 5 && L[0] >= 48 && (L[0] * mm) % 4 == 0 && slab_lds <= 80 * 1024) {
        // slabs of kSlabY whole rows; runs of ZC planes, enough runs for ~2048
        // workgroups, and few enough sites per thread that every 16-bit field
        // stays exact (a site adds at most 12 to a field)
        const int pitch = (4 * nd + 15) & ~15;
        const int ny = (L[1] + kSlabY - 1) / kSlabY;
        const int per_thread = (kSlabY * L[0] + kSlabBlock - 1) / kSlabBlock * mm;  // sites per plane
        const int zc_max = std::max(1, 5000 / per_thread);
        // ~2048 workgroups for large batches, fewer (about 16k sites each)
        // for small ones, whose cost would otherwise be staging and flushes
        const int64_t want = std::min<int64_t>(2048, std::max<int64_t>(1, (int64_t)B * N / 16384));
        int64_t runs = std::max<int64_t>(1, (want + (int64_t)ny * B - 1) / ((int64_t)ny * B));
        int zc = (int)std::min<int64_t>(L[2], std::max<int64_t>(1, (L[2] + runs - 1) / runs));
        zc = std::min(zc, zc_max);
        const int nz = (L[2] + zc - 1) / zc;
        if (B > 65535) return hipErrorInvalidValue;
        // the window, which also holds the final reduction: a row of
        // kMaxShells x KF^2 words per wave and one of totals
        const int kf = K <= 4 ? 4 : 5;
        const size_t red = (size_t)(kSlabBlock / 64 + 1) * kMaxShells * kf * kf * 4;
        const size_t lds = std::max<size_t>((size_t)4 * (kSlabY + 4) * pitch, red);
        const dim3 g((unsigned)ny, (unsigned)nz, (unsigned)B), b(kSlabBlock);
        auto go = [&](const void* kern) {
            (void)hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            void* args[] = {(void*)&occ, (void*)&N, (void*)&L[0], (void*)&L[1], (void*)&L[2], (void*)&K, (void*)&S,
                            (void*)&zc, (void*)&pitch, (void*)&counts};
            return hipLaunchKernel(kern, g, b, args, lds, st);
        };
        hipError_t e;
        if (lattice == SMCX_BCC)
            e = go(kf == 4 ? (const void*)k_pair_counts_slab<SMCX_BCC, 4> : (const void*)k_pair_counts_slab<SMCX_BCC, 5>);
        else
            e = go(kf == 4 ? (const void*)k_pair_counts_slab<SMCX_FCC, 4> : (const void*)k_pair_counts_slab<SMCX_FCC, 5>);
        if (e != hipSuccess) return e;
        return hipGetLastError();
    }
    if (K <= 4) {
        // lanes 64 x 4 cells (16 x 16 for narrow lattices), 16 cells deep;
        // at most 2048 sites per lane between flushes keeps every 16-bit
        // field exact (a site adds at most 24 to a field)
        const int m = lattice == SMCX_BCC ? 2 : 4;
        const bool wide = L[0] >= 48;
        const int TX = wide ? 64 : 16, TY = kBlock / TX;
        const int64_t ntiles = (int64_t)((L[0] + TX - 1) / TX) * ((L[1] + TY - 1) / TY) * ((L[2] + 15) / 16);
        // up to 2048 / (16 m) tiles per workgroup, fewer when the batch has
        // too few tiles to give the chip ~2048 workgroups
        const int64_t tpb_max = 2048 / (m * 16);
        const int tpb = (int)std::max<int64_t>(1, std::min<int64_t>(tpb_max, (ntiles * B + 2047) / 2048));
        const int64_t nbx = (ntiles + tpb - 1) / tpb;
        if (nbx > 0x7fffffff || B > 65535) return hipErrorInvalidValue;
        const dim3 g((unsigned)nbx, (unsigned)B), b(kBlock);
        auto go = [&](auto kern) { hipLaunchKernelGGL(kern, g, b, 0, st, occ, N, L[0], L[1], L[2], K, S, tpb, counts); };
        if (lattice == SMCX_BCC) {
            if (wide) go(k_pair_counts_tiled<SMCX_BCC, 64>); else go(k_pair_counts_tiled<SMCX_BCC, 16>);
        } else {
            if (wide) go(k_pair_counts_tiled<SMCX_FCC, 64>); else go(k_pair_counts_tiled<SMCX_FCC, 16>);
        }
        return hipGetLastError();
    }
    const int64_t ncell = (int64_t)L[0] * L[1] * L[2];
    // <= 2048 sites per lane between flushes keeps the 16-bit fields exact
    const int m = lattice == SMCX_BCC ? 2 : 4;
    const int cells_per_block = kBlock * (2048 / (m * 4));
    const int64_t nbx = (ncell + cells_per_block - 1) / cells_per_block;
    if (nbx > 0x7fffffff || B > 65535) return hipErrorInvalidValue;
    const dim3 g((unsigned)nbx, (unsigned)B), b(kBlock);
    if (lattice == SMCX_BCC) {
        if (K <= 4) hipLaunchKernelGGL((k_pair_counts<SMCX_BCC, 4>), g, b, 0, st, occ, N, L[0], L[1], L[2], K, S, cells_per_block, counts);
        else hipLaunchKernelGGL((k_pair_counts<SMCX_BCC, 8>), g, b, 0, st, occ, N, L[0], L[1], L[2], K, S, cells_per_block, counts);
    } else {
        if (K <= 4) hipLaunchKernelGGL((k_pair_counts<SMCX_FCC, 4>), g, b, 0, st, occ, N, L[0], L[1], L[2], K, S, cells_per_block, counts);
        else hipLaunchKernelGGL((k_pair_counts<SMCX_FCC, 8>), g, b, 0, st, occ, N, L[0], L[1], L[2], K, S, cells_per_block, counts);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Static workspace for smcx_lattice_init_static: a file-scope device array, so
// that a caller that cannot allocate device memory still gets a workspace.
// Every device holds its own copy at its own address, resolved here once per
// device (that device current) with hipGetSymbolAddress; host code passes
// that address on, never the array's name, which in host code is only a
// stand-in for the symbol.
// ---------------------------------------------------------------------------
static __device__ __align__(256) uint8_t scratch[kStaticWorkspaceBytes];

hipError_t static_workspace(void** ptr)
{
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

}  // namespace smcx
