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
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    o0 = c0; o1 = c1; o2 = c2; o3 = c3;
}

template <int NW> struct CounterT;
template <> struct CounterT<1> { using T = uint32_t; static constexpr uint32_t bias = 0x80808080u; };
template <> struct CounterT<2> {
    using T = uint64_t;
    static constexpr uint64_t bias = 0x8080808080808080ull;
};

// Write one species value to a site and to every periodic image of it that
// lies inside the padded copy.
__device__ __forceinline__ void store_site(uint8_t* pad, const RepDev& rep, int m, int x, int y, int z,
                                           int b, uint8_t v)
{
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
            uint8_t* row = pad + ((int64_t)(zs[iz] + kHalo) * rep.prows + (ys[iy] + kHalo)) * rep.prow;
            for (int ix = 0; ix < nx; ++ix) row[m * (xs[ix] + kHalo) + b] = v;
        }
}

// Packed neighbour counters of a basis-B site at LDS byte `base`: A[s] gets
// 1 << (8 * species) per neighbour of shell s.  Offsets are compile-time
// displacements times the launch-uniform window pitches.
template <int LAT, int B, typename CT>
__device__ __forceinline__ void count_uniform(const uint8_t* win, int base, int LP, int PL, int S,
                                              CT (&A)[kMaxShells])
{
    constexpr Geometry G = kGeom[LAT];
#pragma unroll
    for (int s = 0; s < kMaxShells; ++s) {
        CT acc = 0;
        if (s < S) {
#pragma unroll
            for (int n = 0; n < G.Z[s]; ++n) {
                const Nb nb = nb_of(G, B, G.v[s][n][0], G.v[s][n][1], G.v[s][n][2]);
                const int off = nb.dz * PL + nb.dy * LP + G.m * nb.dx + (nb.bt - B);
                acc += (CT)1 << win[base + off];
            }
        }
        A[s] = acc;
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
            for (int n = 0; n < G.Z[s]; ++n) acc += (CT)1 << win[base + offs[j + n]];
        }
        j += G.Z[s];
        A[s] = acc;
    }
}

struct Lds {
    const double* D;
    const int16_t* offP;
    const int32_t* offB;
    const int8_t* pd;
    const uint8_t* mult;
    uint8_t* win;
};

__device__ __forceinline__ Lds lds_ptrs(const SweepArgs& A, uint8_t* smem)
{
    Lds l;
    l.D = (const double*)(smem + A.lds_d);
    l.offP = (const int16_t*)(smem + A.lds_offp);
    l.offB = (const int32_t*)(smem + A.lds_offb);
    l.pd = (const int8_t*)(smem + A.lds_pd);
    l.mult = smem + A.lds_mult;
    l.win = smem + A.lds_win;
    return l;
}

// Copy the launch tables and the replica's partner-image counts into LDS.
template <int LAT>
__device__ void load_tables(const SweepArgs& A, const RepDev& rep, uint8_t* smem)
{
    constexpr int m = kGeom[LAT].m;
    double* D = (double*)(smem + A.lds_d);
    const int nD = A.K * A.K * A.S * A.K;
    for (int i = threadIdx.x; i < nD; i += blockDim.x) D[i] = A.Dtab[i];
    if constexpr (LAT == SMCX_FCC) {
        int16_t* P = (int16_t*)(smem + A.lds_offp);
        const int nP = m * A.Z1 * A.sumZ;
        for (int i = threadIdx.x; i < nP; i += blockDim.x) P[i] = A.offP[i];
    }
    int32_t* Bo = (int32_t*)(smem + A.lds_offb);
    int8_t* pd = (int8_t*)(smem + A.lds_pd);
    for (int i = threadIdx.x; i < m * A.Z1; i += blockDim.x) Bo[i] = A.offB[i];
    for (int i = threadIdx.x; i < 4 * m * A.Z1; i += blockDim.x) pd[i] = A.pdisp[i];
    uint8_t* mu = smem + A.lds_mult;
    for (int i = threadIdx.x; i < kMaxShells * kMaxZ1; i += blockDim.x)
        mu[i] = rep.mult[i / kMaxZ1][i % kMaxZ1];
}

struct TileGeom {
    int w0[3];  // window origin (replica conventional cells, >= -H)
    int n[3];   // window extent
    int gx0;    // first staged byte of each padded row
};

// One lane's trial.  Returns flags: bit0 active, bit1 accepted, bit2 near-tie.
template <int LAT, int NW, int B>
__device__ __forceinline__ int lane_trial(const SweepArgs& A, const RepDev& rep, uint8_t* pad,
                                          const Lds& T, const TileGeom& tg, int r, uint32_t t,
                                          double beta, int ax, int ay, int az)
{
    using CT = typename CounterT<NW>::T;
    constexpr Geometry G = kGeom[LAT];
    constexpr int m = G.m;
    const int LP = A.LP, PL = A.LP * A.WY;
    const uint8_t* win = T.win;
    const int la = ((az - tg.w0[2]) * A.WY + (ay - tg.w0[1])) * LP + (m * (ax + kHalo) + B - tg.gx0);
    const int64_t ia = B + (int64_t)m * (ax + (int64_t)rep.L[0] * (ay + (int64_t)rep.L[1] * az));

    uint32_t w0, w1, w2, w3;
    philox4x32_10((uint32_t)ia, (uint32_t)((uint64_t)ia >> 32), t, (uint32_t)r, (uint32_t)A.seed,
                  (uint32_t)(A.seed >> 32), w0, w1, w2, w3);
    (void)w3;
    const int k = (int)__umulhi(w0, (uint32_t)A.Z1);
    const int p8 = win[la];
    const int offb = T.offB[B * A.Z1 + k];
    const int q8 = win[la + offb];
    if (p8 == q8) return 1;

    CT Ca[kMaxShells], Cb[kMaxShells];
    count_uniform<LAT, B, CT>(win, la, LP, PL, A.S, Ca);
    if constexpr (LAT == SMCX_BCC) {
        // the partner of a BCC site always sits on the other sublattice
        count_uniform<LAT, 1 - B, CT>(win, la + offb, LP, PL, A.S, Cb);
    } else {
        count_table<LAT, CT>(win, la, T.offP + (B * A.Z1 + k) * A.sumZ, A.S, Cb);
    }

    // species were checked < K at init; the clamp keeps table reads in bounds regardless
    const int p = min(p8 >> 3, A.K - 1), q = min(q8 >> 3, A.K - 1);
    const double* Dp = T.D + (size_t)((p * A.K + q) * A.S) * A.K;
    constexpr int KP = NW == 1 ? 4 : 8;
    double dE = 0.0;
#pragma unroll
    for (int s = 0; s < kMaxShells; ++s) {
        if (s < A.S) {
            const CT mu = (CT)T.mult[s * kMaxZ1 + k];
            const CT d = Ca[s] + CounterT<NW>::bias - Cb[s] + (mu << p8) - (mu << q8);
#pragma unroll
            for (int tt = 0; tt < KP; ++tt) {
                if (tt < A.K) {
                    const int c = (int)((d >> (8 * tt)) & 0xFF) - 128;
                    dE = dE + (double)c * Dp[s * A.K + tt];
                }
            }
        }
    }

    bool acc;
    bool tie = false;
    if (dE <= 0.0) {
        acc = true;
    } else {
        const double x = beta * dE;
        const double P = exp(-x);
        const double u = (double)(((uint64_t)w1 << 21) | (uint64_t)(w2 >> 11)) * 0x1p-53;
        acc = u < P;
        tie = fabs(u - P) < 1e-12;
    }
    if (tie) {
        const int slot = atomicAdd(A.tie_count, 1);
        if (slot < A.tie_cap) {
            smcx_tie e;
            e.replica = r;
            e.sweep = t;
            e.site = ia;
            e.decision = acc ? 1 : 0;
            e.pad = 0;
            A.ties[slot] = e;
        }
    }
    if (acc) {
        const int8_t* pd = T.pd + (B * A.Z1 + k) * 4;
        int bx = ax + pd[0], by = ay + pd[1], bz = az + pd[2];
        const int bb = pd[3];
        bx += bx < 0 ? rep.L[0] : (bx >= rep.L[0] ? -rep.L[0] : 0);
        by += by < 0 ? rep.L[1] : (by >= rep.L[1] ? -rep.L[1] : 0);
        bz += bz < 0 ? rep.L[2] : (bz >= rep.L[2] ? -rep.L[2] : 0);
        store_site(pad, rep, m, ax, ay, az, B, (uint8_t)q);
        store_site(pad, rep, m, bx, by, bz, bb, (uint8_t)p);
    }
    return 1 | (acc ? 2 : 0) | (tie ? 4 : 0);
}

template <int LAT, int NW>
__device__ __forceinline__ int lane_dispatch(int b, const SweepArgs& A, const RepDev& rep, uint8_t* pad,
                                             const Lds& T, const TileGeom& tg, int r, uint32_t t,
                                             double beta, int ax, int ay, int az)
{
    if constexpr (LAT == SMCX_BCC) {
        if (b == 0) return lane_trial<LAT, NW, 0>(A, rep, pad, T, tg, r, t, beta, ax, ay, az);
        return lane_trial<LAT, NW, 1>(A, rep, pad, T, tg, r, t, beta, ax, ay, az);
    } else {
        switch (b) {
        case 0: return lane_trial<LAT, NW, 0>(A, rep, pad, T, tg, r, t, beta, ax, ay, az);
        case 1: return lane_trial<LAT, NW, 1>(A, rep, pad, T, tg, r, t, beta, ax, ay, az);
        case 2: return lane_trial<LAT, NW, 2>(A, rep, pad, T, tg, r, t, beta, ax, ay, az);
        default: return lane_trial<LAT, NW, 3>(A, rep, pad, T, tg, r, t, beta, ax, ay, az);
        }
    }
}

// Process one tile of one mini-step: stage the window into LDS, run the
// lanes' trials, add the statistics.  Every thread of the block calls it with
// the same arguments; it starts and ends with a block barrier.
template <int LAT, int NW>
__device__ void run_tile(const SweepArgs& A, const RepDev& rep, int r, int64_t tile, int tau,
                         uint32_t t, double beta, const Lds& T)
{
    constexpr int m = kGeom[LAT].m;
    const int b = tau % m;
    int rest = tau / m;
    const int o[3] = {rest % rep.M[0], (rest / rep.M[0]) % rep.M[1], rest / (rep.M[0] * rep.M[1])};

    const int tx = (int)(tile % rep.ntile[0]);
    const int64_t trest = tile / rep.ntile[0];
    const int ty = (int)(trest % rep.ntile[1]);
    const int tz = (int)(trest / rep.ntile[1]);
    const int c0[3] = {tx * A.T[0], ty * A.T[1], tz * A.T[2]};
    int c1[3];
    const int32_t* org[3];
    org[0] = A.origins + rep.cs_off;
    org[1] = org[0] + rep.nc[0] + 1;
    org[2] = org[1] + rep.nc[1] + 1;
    TileGeom tg;
    bool empty = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        c1[a] = min(c0[a] + A.T[a], rep.nc[a]);
        tg.w0[a] = org[a][c0[a]] + o[a] - kHalo;
        const int w1 = min(org[a][c1[a] - 1] + o[a] + kHalo + 1, rep.L[a] + kHalo);
        tg.n[a] = w1 - tg.w0[a];
        empty |= tg.n[a] <= 0;
    }
    if (empty) return;  // uniform across the block
    tg.gx0 = (m * (tg.w0[0] + kHalo)) & ~15;
    const int gx1 = (m * (tg.w0[0] + tg.n[0] + kHalo) + 15) & ~15;
    const int n16 = (gx1 - tg.gx0) >> 4;

    uint8_t* pad = A.ws + rep.pad_off;
    __syncthreads();  // the previous tile's lanes are done with the window
    {
        // stage: 16-byte loads, species shifted left by 3 (8 * sigma)
        const int per = blockDim.x / n16;
        const int col = threadIdx.x % n16;
        int row = threadIdx.x / n16;
        const int nrows = tg.n[1] * tg.n[2];
        if (row < per) {
            int wy = row % tg.n[1];
            int wz = row / tg.n[1];
            for (; row < nrows; row += per) {
                const uint8_t* src =
                    pad + ((int64_t)(tg.w0[2] + wz + kHalo) * rep.prows + (tg.w0[1] + wy + kHalo)) * rep.prow +
                    tg.gx0 + 16 * col;
                uint4 v = *(const uint4*)src;
                v.x = (v.x << 3) & 0xF8F8F8F8u;
                v.y = (v.y << 3) & 0xF8F8F8F8u;
                v.z = (v.z << 3) & 0xF8F8F8F8u;
                v.w = (v.w << 3) & 0xF8F8F8F8u;
                *(uint4*)(T.win + (wz * A.WY + wy) * A.LP + 16 * col) = v;
                wy += per;
                while (wy >= tg.n[1]) {
                    wy -= tg.n[1];
                    ++wz;
                }
            }
        }
    }
    __syncthreads();

    const int l = threadIdx.x;
    const int lx = l % A.T[0];
    const int ly = (l / A.T[0]) % A.T[1];
    const int lz = l / (A.T[0] * A.T[1]);
    const int cx = c0[0] + lx, cy = c0[1] + ly, cz = c0[2] + lz;
    bool active = lz < A.T[2] && cx < c1[0] && cy < c1[1] && cz < c1[2];
    int ax = 0, ay = 0, az = 0;
    if (active) {
        ax = org[0][cx] + o[0];
        ay = org[1][cy] + o[1];
        az = org[2][cz] + o[2];
        active = ax < org[0][cx + 1] && ay < org[1][cy + 1] && az < org[2][cz + 1];
    }
    int f = 0;
    if (active) f = lane_dispatch<LAT, NW>(b, A, rep, pad, T, tg, r, t, beta, ax, ay, az);

    const uint64_t att = __ballot(f & 1), accm = __ballot(f & 2), tiem = __ballot(f & 4);
    if ((threadIdx.x & 63) == 0 && att) {
        unsigned long long* st = (unsigned long long*)(A.stats + 3 * (int64_t)r);
        atomicAdd(st + 0, (unsigned long long)__popcll(att));
        if (accm) atomicAdd(st + 1, (unsigned long long)__popcll(accm));
        if (tiem) atomicAdd(st + 2, (unsigned long long)__popcll(tiem));
    }
}

// ---------------------------------------------------------------------------
// Stream mode: one launch per mini-step g, one workgroup per tile over all
// replicas.  Logical tiles are handed out so that consecutive tiles (which
// share halo rows) run on the same XCD: hardware workgroup i goes to XCD
// i % 8, so logical tile = (i % 8) * xcd_per + i / 8.
// ---------------------------------------------------------------------------
template <int LAT, int NW>
__global__ __launch_bounds__(kBlock) void k_ministep(SweepArgs A)
{
    extern __shared__ __align__(16) uint8_t smem[];
    const int64_t i = blockIdx.x;
    int64_t tile = (i % 8) * (int64_t)A.xcd_per + i / 8;
    int r;
    if (A.only_rep >= 0) {
        r = A.only_rep;
        if (tile >= A.reps[r].ntiles) return;
    } else {
        if (tile >= A.tile_off[A.R]) return;
        int lo = 0, hi = A.R - 1;  // last r with tile_off[r] <= tile
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (A.tile_off[mid] <= tile) lo = mid; else hi = mid - 1;
        }
        r = lo;
        tile -= A.tile_off[r];
    }
    const RepDev& rep = A.reps[r];
    if (A.g >= rep.nA) return;
    load_tables<LAT>(A, rep, smem);
    const Lds T = lds_ptrs(A, smem);
    __syncthreads();
    const double beta = A.beta[r];  // host passes the sweep's row
    run_tile<LAT, NW>(A, rep, r, tile, A.g, A.first_sweep, beta, T);
}

// ---------------------------------------------------------------------------
// Persistent mode: one workgroup per replica runs every sweep and mini-step;
// the replica's tiles of one mini-step are processed one after another and
// block barriers order the mini-steps (all writes of a replica come from its
// own workgroup).
// ---------------------------------------------------------------------------
template <int LAT, int NW>
__global__ __launch_bounds__(kBlock) void k_persistent(SweepArgs A)
{
    extern __shared__ __align__(16) uint8_t smem[];
    const int r = blockIdx.x;
    const RepDev& rep = A.reps[r];
    load_tables<LAT>(A, rep, smem);
    const Lds T = lds_ptrs(A, smem);
    __syncthreads();
    const uint32_t first = A.sweep_counter ? *A.sweep_counter : A.first_sweep;
    for (int js = 0; js < A.n_sweeps; ++js) {
        const uint32_t t = first + (uint32_t)js;
        const double beta = A.beta[(int64_t)js * A.beta_stride + r];
        const int tau_end = min(A.tau_end, rep.nA);
        for (int tau = A.tau_begin; tau < tau_end; ++tau)
            for (int64_t tile = 0; tile < rep.ntiles; ++tile)
                run_tile<LAT, NW>(A, rep, r, tile, tau, t, beta, T);
    }
}

__global__ void k_advance_counter(uint32_t* counter, uint32_t n)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *counter += n;
}

// Natural layout -> padded copy (all halo images).
template <int M>
__global__ void k_pack(const uint8_t* occ, uint8_t* ws, const RepDev* reps, int r)
{
    const RepDev& rep = reps[r];
    uint8_t* pad = ws + rep.pad_off;
    const uint8_t* o = occ + rep.occ_off;
    const int64_t ncell = (int64_t)rep.L[0] * rep.L[1] * rep.L[2];
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < ncell;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(c % rep.L[0]);
        const int64_t cr = c / rep.L[0];
        const int y = (int)(cr % rep.L[1]);
        const int z = (int)(cr / rep.L[1]);
#pragma unroll
        for (int b = 0; b < M; ++b) store_site(pad, rep, M, x, y, z, b, o[M * c + b]);
    }
}

// Padded copy interior -> natural layout.
template <int M>
__global__ void k_unpack(uint8_t* occ, const uint8_t* ws, const RepDev* reps, int r)
{
    const RepDev& rep = reps[r];
    const uint8_t* pad = ws + rep.pad_off;
    uint8_t* o = occ + rep.occ_off;
    const int64_t ncell = (int64_t)rep.L[0] * rep.L[1] * rep.L[2];
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < ncell;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(c % rep.L[0]);
        const int64_t cr = c / rep.L[0];
        const int y = (int)(cr % rep.L[1]);
        const int z = (int)(cr / rep.L[1]);
        const uint8_t* row = pad + ((int64_t)(z + kHalo) * rep.prows + (y + kHalo)) * rep.prow + M * (x + kHalo);
#pragma unroll
        for (int b = 0; b < M; ++b) o[M * c + b] = row[b];
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
// Host-side launchers
// ---------------------------------------------------------------------------
template <int LAT, int NW>
static hipError_t launch_sweep_t(bool persistent, dim3 grid, size_t lds, hipStream_t st, const SweepArgs& a)
{
    if (persistent) {
        hipLaunchKernelGGL((k_persistent<LAT, NW>), grid, dim3(kBlock), lds, st, a);
    } else {
        hipLaunchKernelGGL((k_ministep<LAT, NW>), grid, dim3(kBlock), lds, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_sweep(int lattice, int K, bool persistent, dim3 grid, size_t lds, hipStream_t st,
                        const SweepArgs& a)
{
    const int nw = K <= 4 ? 1 : 2;
    if (lattice == SMCX_BCC)
        return nw == 1 ? launch_sweep_t<SMCX_BCC, 1>(persistent, grid, lds, st, a)
                       : launch_sweep_t<SMCX_BCC, 2>(persistent, grid, lds, st, a);
    return nw == 1 ? launch_sweep_t<SMCX_FCC, 1>(persistent, grid, lds, st, a)
                   : launch_sweep_t<SMCX_FCC, 2>(persistent, grid, lds, st, a);
}

hipError_t set_sweep_lds_limit(int lattice, int K, size_t lds)
{
    const int nw = K <= 4 ? 1 : 2;
    const void* f1;
    const void* f2;
    if (lattice == SMCX_BCC) {
        f1 = nw == 1 ? (const void*)k_ministep<SMCX_BCC, 1> : (const void*)k_ministep<SMCX_BCC, 2>;
        f2 = nw == 1 ? (const void*)k_persistent<SMCX_BCC, 1> : (const void*)k_persistent<SMCX_BCC, 2>;
    } else {
        f1 = nw == 1 ? (const void*)k_ministep<SMCX_FCC, 1> : (const void*)k_ministep<SMCX_FCC, 2>;
        f2 = nw == 1 ? (const void*)k_persistent<SMCX_FCC, 1> : (const void*)k_persistent<SMCX_FCC, 2>;
    }
    hipError_t e = hipFuncSetAttribute(f1, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(f2, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t launch_pack(int lattice, bool unpack, uint8_t* occ, uint8_t* ws, const RepDev* reps, int r,
                       int64_t ncell, hipStream_t st)
{
    int64_t nb = (ncell + kBlock - 1) / kBlock;
    if (nb > 65536) nb = 65536;
    if (nb < 1) nb = 1;
    const dim3 g((unsigned)nb), b(kBlock);
    if (lattice == SMCX_BCC) {
        if (unpack) hipLaunchKernelGGL(k_unpack<2>, g, b, 0, st, occ, ws, reps, r);
        else hipLaunchKernelGGL(k_pack<2>, g, b, 0, st, occ, ws, reps, r);
    } else {
        if (unpack) hipLaunchKernelGGL(k_unpack<4>, g, b, 0, st, occ, ws, reps, r);
        else hipLaunchKernelGGL(k_pack<4>, g, b, 0, st, occ, ws, reps, r);
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

}  // namespace smcx
