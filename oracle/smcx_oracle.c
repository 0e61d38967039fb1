/*
 * smcx_oracle.c -- plain, slow, sequential CPU oracle for link-cell parallel
 * canonical swap Metropolis Monte Carlo with a multi-shell effective pair
 * interaction (EPI) energy on BCC / FCC lattices.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference that the HIP path is
 * checked against.  It shares no code, header, table or constant generator
 * with the HIP library, and nothing in the product path may link or call it:
 * only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark use it.
 *
 * Arithmetic: IEEE binary64, compiled with -ffp-contract=off so that every
 * multiply and add is rounded separately, in the order written here.
 *
 * What it follows (paper: "Revealing Nanostructures in High-Entropy Alloys
 * via Machine-Learning Accelerated Scalable Monte Carlo Simulation"):
 *   - sites labelled by (link cell i_C, position in the cell i_A); a sweep is
 *     n_A sequential mini-steps, each holding one trial per link cell
 *     (Results sec. "Performance of the SMC-X algorithm"; Methods sec.
 *     "Implementation of SMC-GPU", link-cell bullet; Fig. 7 caption);
 *   - two trials are independent when neither move changes what the other
 *     reads (the LIZ / LIZ+ argument, same Results section, Fig. 1c);
 *   - canonical swap move with a nearest-neighbour partner and the Metropolis
 *     acceptance min(1, exp(-beta dE)) (Supplementary "Monte Carlo Simulation
 *     Algorithms", acceptance equation; a sweep is one trial per site);
 *   - EPI energy: pair interactions of each site with its neighbours shell by
 *     shell (Methods sec. "The EPI and qSRO model", Eq. Linear_EPI and
 *     Eq. Total_EPI); for a pair model the energy change of a swap is twice
 *     the change of the two local energies (same section, text after
 *     Eq. Total_EPI);
 *   - neighbours found by index arithmetic from a list of relative positions
 *     (Methods, "Search neighbors" bullet).
 * Where the paper is silent the conventions are (each is a reading, listed
 * with its reason in the design notes):
 *   E = 1/2 sum_i sum_s sum_{d in D_s} V_s[sigma_i][sigma_{i+d}] (directed
 *   offset-table definition, duplicate periodic images counted with
 *   multiplicity); periodic boundaries; D_s sorted lexicographically; partner
 *   k = floor(w0 * Z_1 / 2^32); Philox4x32-10 keyed by the seed with counter
 *   (site_lo, site_hi, sweep, replica); u from 53 bits of (w1, w2); a trial
 *   whose partner has the same species is attempted but not accepted;
 *   accept when dE <= 0, else when u < exp(-beta dE) strictly; a decision
 *   with |u - exp(-beta dE)| < 1e-12 is a near-tie, logged, and replaced by a
 *   replayed decision when one is supplied.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXS 4
#define OR_MAXZ 24
#define OR_MAXK 8
#define OR_BCC 0
#define OR_FCC 1

/* error codes */
#define OR_OK 0
#define OR_EARG (-1)

/* Near-tie record: 24 bytes, {replica, sweep, site, decision, pad}. */
typedef struct {
    int32_t replica;
    uint32_t sweep;
    int64_t site;
    int32_t decision;
    int32_t pad;
} or_tie;

/* One trial as executed, in execution order (single-thread runs only). */
typedef struct {
    int64_t a;       /* active site */
    int64_t b;       /* partner site */
    double dE;       /* energy change (0 when p == q) */
    int32_t k;       /* partner direction index in D_1 */
    int32_t accepted;
} or_trace;

/* ------------------------------------------------------------------------ */
/* Geometry: conventional cubic cell with m basis sites, positions in units  */
/* of half the lattice constant.                                             */
/* ------------------------------------------------------------------------ */

typedef struct {
    int m;
    int basis[4][3];
} or_lat;

static int lat_get(int lattice, or_lat *lt)
{
    memset(lt, 0, sizeof(*lt));
    if (lattice == OR_BCC) {
        /* body-centred cubic: (0,0,0) and (a/2)(1,1,1) */
        lt->m = 2;
        lt->basis[1][0] = 1; lt->basis[1][1] = 1; lt->basis[1][2] = 1;
        return OR_OK;
    }
    if (lattice == OR_FCC) {
        /* face-centred cubic: (0,0,0) and the three face centres */
        lt->m = 4;
        lt->basis[1][0] = 1; lt->basis[1][1] = 1;
        lt->basis[2][0] = 1; lt->basis[2][2] = 1;
        lt->basis[3][1] = 1; lt->basis[3][2] = 1;
        return OR_OK;
    }
    return OR_EARG;
}

static int pmod(int a, int n) { int r = a % n; return r < 0 ? r + n : r; }

/* A vector is a lattice vector when its parity pattern is that of a basis
 * position (all basis positions are measured from basis 0 at the origin). */
static int is_lattice_vector(const or_lat *lt, int dx, int dy, int dz)
{
    for (int b = 0; b < lt->m; ++b)
        if (pmod(dx, 2) == lt->basis[b][0] && pmod(dy, 2) == lt->basis[b][1] &&
            pmod(dz, 2) == lt->basis[b][2])
            return 1;
    return 0;
}

/*
 * Coordination shells: D_s = all lattice vectors whose squared length is the
 * s-th smallest non-zero value, sorted lexicographically by (dx, dy, dz).
 * Z[s] receives |D_s|; d receives the vectors, row s at d[s*24*3].
 * Returns OR_OK or OR_EARG.  (Neighbour list of relative positions, Methods
 * "Search neighbors" bullet.)
 */
int or_shells(int lattice, int S, int32_t *Z, int32_t *d)
{
    or_lat lt;
    if (lat_get(lattice, &lt) != OR_OK || S < 1 || S > OR_MAXS) return OR_EARG;
    /* distinct squared lengths, ascending */
    int r2[OR_MAXS];
    int nr = 0;
    for (int target = 1; nr < S && target < 64; ++target) {
        int found = 0;
        for (int dx = -4; dx <= 4 && !found; ++dx)
            for (int dy = -4; dy <= 4 && !found; ++dy)
                for (int dz = -4; dz <= 4 && !found; ++dz)
                    if (dx * dx + dy * dy + dz * dz == target && is_lattice_vector(&lt, dx, dy, dz))
                        found = 1;
        if (found) r2[nr++] = target;
    }
    if (nr < S) return OR_EARG;
    for (int s = 0; s < S; ++s) {
        int n = 0;
        /* nested ascending loops produce lexicographic order directly */
        for (int dx = -4; dx <= 4; ++dx)
            for (int dy = -4; dy <= 4; ++dy)
                for (int dz = -4; dz <= 4; ++dz)
                    if (dx * dx + dy * dy + dz * dz == r2[s] && is_lattice_vector(&lt, dx, dy, dz)) {
                        if (n >= OR_MAXZ) return OR_EARG;
                        int32_t *v = d + ((size_t)s * OR_MAXZ + n) * 3;
                        v[0] = dx; v[1] = dy; v[2] = dz;
                        ++n;
                    }
        Z[s] = n;
    }
    return OR_OK;
}

/*
 * Smallest link-cell edge (in conventional cells) for which trials in one
 * mini-step are independent.  A pair-model trial at a reads sites within
 * 1 + c_max half-units of a (the partner is within 1, its neighbours within
 * c_max of it) and writes sites within 1 of its own site; the LIZ form
 * (nonlinear local-energy models, liz != 0) reads within 1 + 2 c_max.  Two
 * active sites of one mini-step are at least 2*ell half-units apart on some
 * axis, so the condition is 2*ell > 1 + reach.  c_max is the largest |component|
 * over the shells in use.  (Link-cell size must exceed the interaction range,
 * Methods, link-cell bullet; LIZ / LIZ+ definition, Results, Fig. 1c.)
 */
int or_lmin(int lattice, int S, int liz)
{
    int32_t Z[OR_MAXS], d[OR_MAXS * OR_MAXZ * 3];
    if (or_shells(lattice, S, Z, d) != OR_OK) return OR_EARG;
    int cmax = 0;
    for (int s = 0; s < S; ++s)
        for (int n = 0; n < Z[s]; ++n)
            for (int a = 0; a < 3; ++a) {
                int c = abs(d[(s * OR_MAXZ + n) * 3 + a]);
                if (c > cmax) cmax = c;
            }
    int reach = liz ? 1 + 2 * cmax : 1 + cmax;
    int ell = 1;
    while (!(2 * ell > 1 + reach)) ++ell;
    return ell;
}

/* Default per-axis partition of L conventional cells into cells of edge
 * about ell: n = max(1, floor(L/ell)) cells, sizes floor(L/n) + [j < L mod n].
 * Writes n sizes and returns n. */
int or_partition(int L, int ell, int32_t *sizes)
{
    if (L < 1 || ell < 1) return OR_EARG;
    int n = L / ell;
    if (n < 1) n = 1;
    for (int j = 0; j < n; ++j) sizes[j] = L / n + (j < L % n ? 1 : 0);
    return n;
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): a 4x32-bit counter is  */
/* passed through 10 rounds of a multiply/xor S-box keyed by a 2x32-bit key  */
/* that is bumped by the Weyl constants between rounds.                      */
/* ------------------------------------------------------------------------ */

void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        if (round < 9) { k0 += W0; k1 += W1; }
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------ */
/* Lattice state                                                             */
/* ------------------------------------------------------------------------ */

typedef struct {
    or_lat lt;
    int L[3];
    int K, S;
    int Z[OR_MAXS];
    int d[OR_MAXS][OR_MAXZ][3];
    int64_t N;
} or_sys;

static int sys_init(or_sys *sy, int lattice, const int32_t L[3], int K, int S)
{
    memset(sy, 0, sizeof(*sy));
    if (lat_get(lattice, &sy->lt) != OR_OK) return OR_EARG;
    if (K < 2 || K > OR_MAXK || S < 1 || S > OR_MAXS) return OR_EARG;
    for (int a = 0; a < 3; ++a) {
        if (L[a] < 1) return OR_EARG;
        sy->L[a] = L[a];
    }
    sy->K = K;
    sy->S = S;
    int32_t Z[OR_MAXS], d[OR_MAXS * OR_MAXZ * 3];
    if (or_shells(lattice, S, Z, d) != OR_OK) return OR_EARG;
    for (int s = 0; s < S; ++s) {
        sy->Z[s] = Z[s];
        for (int n = 0; n < Z[s]; ++n)
            for (int a = 0; a < 3; ++a) sy->d[s][n][a] = d[(s * OR_MAXZ + n) * 3 + a];
    }
    /* reject a lattice on which some neighbour vector maps a site onto itself */
    for (int s = 0; s < S; ++s)
        for (int n = 0; n < Z[s]; ++n)
            if (pmod(sy->d[s][n][0], 2 * L[0]) == 0 && pmod(sy->d[s][n][1], 2 * L[1]) == 0 &&
                pmod(sy->d[s][n][2], 2 * L[2]) == 0)
                return OR_EARG;
    sy->N = (int64_t)sy->lt.m * L[0] * L[1] * L[2];
    return OR_OK;
}

/* site index i = b + m*(x + Lx*(y + Ly*z)) */
static int64_t site_index(const or_sys *sy, int b, int x, int y, int z)
{
    return b + (int64_t)sy->lt.m * (x + (int64_t)sy->L[0] * (y + (int64_t)sy->L[1] * z));
}

static void site_pos(const or_sys *sy, int64_t i, int h[3])
{
    int m = sy->lt.m;
    int b = (int)(i % m);
    int64_t c = i / m;
    int x = (int)(c % sy->L[0]);
    int y = (int)((c / sy->L[0]) % sy->L[1]);
    int z = (int)(c / ((int64_t)sy->L[0] * sy->L[1]));
    h[0] = 2 * x + sy->lt.basis[b][0];
    h[1] = 2 * y + sy->lt.basis[b][1];
    h[2] = 2 * z + sy->lt.basis[b][2];
}

/* site at half-unit position h + v, periodic in all three directions */
static int64_t site_at(const or_sys *sy, const int h[3], const int v[3])
{
    int g[3];
    for (int a = 0; a < 3; ++a) g[a] = pmod(h[a] + v[a], 2 * sy->L[a]);
    int b = -1;
    for (int bb = 0; bb < sy->lt.m; ++bb)
        if ((g[0] & 1) == sy->lt.basis[bb][0] && (g[1] & 1) == sy->lt.basis[bb][1] &&
            (g[2] & 1) == sy->lt.basis[bb][2])
            b = bb;
    /* v is a lattice vector, so the parity pattern always matches a basis site */
    return site_index(sy, b, (g[0] - sy->lt.basis[b][0]) / 2, (g[1] - sy->lt.basis[b][1]) / 2,
                      (g[2] - sy->lt.basis[b][2]) / 2);
}

/* ------------------------------------------------------------------------ */
/* Pair counts, energy and short-range order                                 */
/* ------------------------------------------------------------------------ */

/*
 * Directed pair counts C[s][k][l] = #{(i, d in D_s): sigma_i = k,
 * sigma_{i+d} = l}.  These are the per-shell pair numbers n_m^{pp'} of the
 * EPI features (Methods, "The EPI and qSRO model", the definition of the
 * pair fractions pi_m^{pp'}), summed over all sites.
 */
int or_pair_counts(int lattice, const int32_t L[3], int K, int S, const uint8_t *occ, int64_t *C)
{
    or_sys sy;
    if (sys_init(&sy, lattice, L, K, S) != OR_OK) return OR_EARG;
    memset(C, 0, sizeof(int64_t) * (size_t)S * K * K);
    for (int64_t i = 0; i < sy.N; ++i) {
        if (occ[i] >= K) return OR_EARG;
        int h[3];
        site_pos(&sy, i, h);
        for (int s = 0; s < S; ++s)
            for (int n = 0; n < sy.Z[s]; ++n) {
                int64_t j = site_at(&sy, h, sy.d[s][n]);
                C[((size_t)s * K + occ[i]) * K + occ[j]] += 1;
            }
    }
    return OR_OK;
}

/* The same counts with the sites split over nthreads OpenMP threads, each
 * counting its own contiguous range into its own table; the tables are then
 * added.  Integer sums, so the result is that of or_pair_counts exactly (for
 * the billion-site lattices, where one thread takes minutes). */
int or_pair_counts_threads(int lattice, const int32_t L[3], int K, int S, const uint8_t *occ, int64_t *C,
                           int32_t nthreads)
{
    or_sys sy;
    if (sys_init(&sy, lattice, L, K, S) != OR_OK || nthreads < 1) return OR_EARG;
    const size_t nC = (size_t)S * K * K;
    int64_t *part = (int64_t *)calloc((size_t)nthreads * nC, sizeof(int64_t));
    if (!part) return OR_EARG;
    int bad = 0;
#pragma omp parallel num_threads(nthreads) reduction(| : bad)
    {
        const int th = omp_get_thread_num(), nth = omp_get_num_threads();
        const int64_t lo = sy.N * th / nth, hi = sy.N * (th + 1) / nth;
        int64_t *Ct = part + (size_t)th * nC;
        for (int64_t i = lo; i < hi; ++i) {
            if (occ[i] >= K) {
                bad = 1;
                break;
            }
            int h[3];
            site_pos(&sy, i, h);
            for (int s = 0; s < S; ++s)
                for (int n = 0; n < sy.Z[s]; ++n) {
                    int64_t j = site_at(&sy, h, sy.d[s][n]);
                    Ct[((size_t)s * K + occ[i]) * K + occ[j]] += 1;
                }
        }
    }
    memset(C, 0, sizeof(int64_t) * nC);
    for (int t = 0; t < nthreads; ++t)
        for (size_t x = 0; x < nC; ++x) C[x] += part[(size_t)t * nC + x];
    free(part);
    return bad ? OR_EARG : OR_OK;
}

/* E = 1/2 sum_{s,k,l} C[s][k][l] V[s][k][l], accumulated s, k, l ascending.
 * (Eq. Total_EPI: the total energy is linear in the pair counts.) */
double or_energy(int K, int S, const int64_t *C, const double *V)
{
    double acc = 0.0;
    for (int s = 0; s < S; ++s)
        for (int k = 0; k < K; ++k)
            for (int l = 0; l < K; ++l) {
                size_t idx = ((size_t)s * K + k) * K + l;
                acc = acc + (double)C[idx] * V[idx];
            }
    return 0.5 * acc;
}

/* Warren-Cowley short-range order from directed counts:
 * alpha_s[k][l] = 1 - C[s][k][l] N / (Z_s N_k N_l).  Species counts N_k are
 * taken from the row sums of shell 0, sum_l C[0][k][l] = Z_0 N_k.  Returns
 * OR_EARG when some species is absent. */
int or_sro(int K, int S, const int32_t *Z, const int64_t *C, double *alpha)
{
    int64_t Nk[OR_MAXK];
    int64_t N = 0;
    for (int k = 0; k < K; ++k) {
        int64_t row = 0;
        for (int l = 0; l < K; ++l) row += C[(size_t)k * K + l];
        if (row % Z[0] != 0) return OR_EARG;
        Nk[k] = row / Z[0];
        if (Nk[k] == 0) return OR_EARG;
        N += Nk[k];
    }
    for (int s = 0; s < S; ++s)
        for (int k = 0; k < K; ++k)
            for (int l = 0; l < K; ++l) {
                size_t idx = ((size_t)s * K + k) * K + l;
                alpha[idx] = 1.0 - ((double)C[idx] * (double)N) /
                                       (((double)Z[s] * (double)Nk[k]) * (double)Nk[l]);
            }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* One swap trial                                                            */
/* ------------------------------------------------------------------------ */

/* Energy change of swapping the species of a and of its partner in
 * direction D_1[k].  n_a[s][t] counts neighbours of a in shell s with species
 * t, over every d with a+d != b (by site index); n_b likewise with b+d != a.
 * dE = sum_s sum_t (n_a - n_b)[s][t] * (V_s[q][t] - V_s[p][t]), s and t
 * ascending, each operation rounded separately.  The a-b bond itself is
 * unchanged by the swap when V is symmetric and is therefore left out.  This
 * is the "twice the change of the two local energies" rule of the pair
 * model (Methods, "The EPI and qSRO model"). */
static double trial_dE(const or_sys *sy, const uint8_t *occ, const double *V, int64_t a, int64_t b)
{
    int K = sy->K, S = sy->S;
    int ha[3], hb[3];
    site_pos(sy, a, ha);
    site_pos(sy, b, hb);
    int p = occ[a], q = occ[b];
    int na[OR_MAXS][OR_MAXK], nb[OR_MAXS][OR_MAXK];
    memset(na, 0, sizeof(na));
    memset(nb, 0, sizeof(nb));
    for (int s = 0; s < S; ++s)
        for (int n = 0; n < sy->Z[s]; ++n) {
            int64_t ja = site_at(sy, ha, sy->d[s][n]);
            if (ja != b) na[s][occ[ja]] += 1;
            int64_t jb = site_at(sy, hb, sy->d[s][n]);
            if (jb != a) nb[s][occ[jb]] += 1;
        }
    double dE = 0.0;
    for (int s = 0; s < S; ++s)
        for (int t = 0; t < K; ++t) {
            double dv = V[((size_t)s * K + q) * K + t] - V[((size_t)s * K + p) * K + t];
            dE = dE + (double)(na[s][t] - nb[s][t]) * dv;
        }
    return dE;
}

/* ------------------------------------------------------------------------ */
/* qSRO model: a nonlinear local energy                                      */
/* ------------------------------------------------------------------------ */

/*
 * qSRO local energy of site i with species p (Methods, "The EPI and qSRO
 * model", Eq. quadratic_local_SRO): the pair fractions of the local
 * environment, pi_m^{p t} = n_i[m][t] / Z_m (centre-neighbour pairs of shell
 * m), enter linearly with V_m[p][t] and, for the same-species pair, squared
 * with W_m[p]:
 *   E_i = sum_m sum_t V_m[p][t] (n_i[m][t] / Z_m) + sum_m W_m[p] (n_i[m][p] / Z_m)^2,
 * in that order (m, then t), each quotient, product and sum rounded.
 */
static double qsro_site(const or_sys *sy, const uint8_t *occ, const double *V, const double *W, int64_t i)
{
    int K = sy->K, S = sy->S;
    int h[3];
    site_pos(sy, i, h);
    int n[OR_MAXS][OR_MAXK];
    memset(n, 0, sizeof(n));
    for (int s = 0; s < S; ++s)
        for (int k = 0; k < sy->Z[s]; ++k) n[s][occ[site_at(sy, h, sy->d[s][k])]] += 1;
    int p = occ[i];
    double acc = 0.0;
    for (int s = 0; s < S; ++s)
        for (int t = 0; t < K; ++t) acc = acc + V[((size_t)s * K + p) * K + t] * ((double)n[s][t] / (double)sy->Z[s]);
    for (int s = 0; s < S; ++s) {
        double f = (double)n[s][p] / (double)sy->Z[s];
        acc = acc + W[(size_t)s * K + p] * (f * f);
    }
    return acc;
}

/* Displacements (half units, from the active site a) of every site whose
 * qSRO local energy a swap of a with its partner in direction D_1[k] can
 * change: a, the partner, and every shell neighbour of either; without
 * duplicates, in lexicographic (x, y, z) order.  Returns the count. */
#define OR_MAXAFF 256
static int qsro_affected(const or_sys *sy, int k, int (*v)[3])
{
    int n = 0;
    int cand[2 + 2 * OR_MAXS * OR_MAXZ][3];
    const int *ab = sy->d[0][k];
    cand[n][0] = cand[n][1] = cand[n][2] = 0;
    ++n;
    for (int a = 0; a < 3; ++a) cand[n][a] = ab[a];
    ++n;
    for (int s = 0; s < sy->S; ++s)
        for (int j = 0; j < sy->Z[s]; ++j) {
            for (int a = 0; a < 3; ++a) cand[n][a] = sy->d[s][j][a];
            ++n;
            for (int a = 0; a < 3; ++a) cand[n][a] = ab[a] + sy->d[s][j][a];
            ++n;
        }
    int m = 0;
    for (int i = 0; i < n; ++i) {
        int dup = 0;
        for (int j = 0; j < m && !dup; ++j)
            dup = v[j][0] == cand[i][0] && v[j][1] == cand[i][1] && v[j][2] == cand[i][2];
        if (dup) continue;
        /* insert in lexicographic order */
        int at = m;
        while (at > 0 && (v[at - 1][0] > cand[i][0] ||
                          (v[at - 1][0] == cand[i][0] && (v[at - 1][1] > cand[i][1] ||
                                                          (v[at - 1][1] == cand[i][1] && v[at - 1][2] > cand[i][2]))))) {
            for (int a = 0; a < 3; ++a) v[at][a] = v[at - 1][a];
            --at;
        }
        for (int a = 0; a < 3; ++a) v[at][a] = cand[i][a];
        ++m;
    }
    return m;
}

/* qSRO energy change of swapping a with its partner b = a + D_1[k]: the
 * local energies of the affected sites before and after the swap (computed
 * on the swapped occupancy, which is then restored), summed as
 * dE = dE + (after_j - before_j) over the affected set in its order.  The
 * paper's rule for models beyond pairs: add up the local energies of every
 * site within the interaction zone (Methods, text before
 * Eq. quadratic_local_SRO). */
static double qsro_dE(const or_sys *sy, uint8_t *occ, const double *V, const double *W, int64_t a, int64_t b, int k)
{
    int v[OR_MAXAFF][3];
    int n = qsro_affected(sy, k, v);
    int ha[3];
    site_pos(sy, a, ha);
    int64_t js[OR_MAXAFF];
    double before[OR_MAXAFF];
    for (int i = 0; i < n; ++i) {
        js[i] = site_at(sy, ha, v[i]);
        before[i] = qsro_site(sy, occ, V, W, js[i]);
    }
    uint8_t p = occ[a], q = occ[b];
    occ[a] = q;
    occ[b] = p;
    double dE = 0.0;
    for (int i = 0; i < n; ++i) dE = dE + (qsro_site(sy, occ, V, W, js[i]) - before[i]);
    occ[a] = p;
    occ[b] = q;
    return dE;
}

/* The 53-bit uniform of a trial or exchange: (w1 2^21 + floor(w2 / 2^11)) 2^-53. */
static double u53(const uint32_t w[4])
{
    return (double)(((uint64_t)w[1] << 21) | (uint64_t)(w[2] >> 11)) * 0x1p-53;
}

typedef struct {
    const or_tie *replay;
    int32_t n_replay;
} or_replay;

static int replay_lookup(const or_replay *rp, int32_t r, uint32_t t, int64_t a, int *decision)
{
    for (int32_t i = 0; i < rp->n_replay; ++i)
        if (rp->replay[i].replica == r && rp->replay[i].sweep == t && rp->replay[i].site == a) {
            *decision = rp->replay[i].decision;
            return 1;
        }
    return 0;
}

/* Result flags of one trial */
#define TR_ACCEPTED 1
#define TR_TIE 2

/*
 * One canonical swap trial at site a during sweep t of replica r
 * (Supplementary, "Monte Carlo Simulation Algorithms"): a uniform nearest
 * neighbour partner, Metropolis acceptance, swap on acceptance.
 */
static int do_trial(const or_sys *sy, uint8_t *occ, const double *V, const double *W, uint64_t seed, uint32_t r,
                    uint32_t t, int64_t a, double beta, const or_replay *rp, or_trace *tr)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {(uint32_t)a, (uint32_t)((uint64_t)a >> 32), t, r};
    uint32_t w[4];
    or_philox4x32_10(ctr, key, w);
    int k = (int)(((uint64_t)w[0] * (uint64_t)sy->Z[0]) >> 32);
    int ha[3];
    site_pos(sy, a, ha);
    int64_t b = site_at(sy, ha, sy->d[0][k]);
    int p = occ[a], q = occ[b];
    int flags = 0;
    double dE = 0.0;
    if (p != q) {
        dE = W ? qsro_dE(sy, occ, V, W, a, b, k) : trial_dE(sy, occ, V, a, b);
        int accept;
        if (dE <= 0.0) {
            accept = 1;
        } else {
            double x = beta * dE;
            double P = exp(-x);
            double u = u53(w);
            accept = u < P;
            if (fabs(u - P) < 1e-12) {
                flags |= TR_TIE;
                int dec;
                if (rp && replay_lookup(rp, (int32_t)r, t, a, &dec)) accept = dec;
            }
        }
        if (accept) {
            occ[a] = (uint8_t)q;
            occ[b] = (uint8_t)p;
            flags |= TR_ACCEPTED;
        }
    }
    if (tr) {
        tr->a = a;
        tr->b = b;
        tr->dE = dE;
        tr->k = k;
        tr->accepted = (flags & TR_ACCEPTED) ? 1 : 0;
    }
    return flags;
}

/* Energy change of one proposed swap (a, D_1[k]) without applying it; 0 when
 * the species are equal.  Exposed for tests. */
int or_delta_e(int lattice, const int32_t L[3], int K, int S, const uint8_t *occ, const double *V,
               int64_t a, int32_t k, double *dE, int64_t *partner)
{
    or_sys sy;
    if (sys_init(&sy, lattice, L, K, S) != OR_OK) return OR_EARG;
    if (a < 0 || a >= sy.N || k < 0 || k >= sy.Z[0]) return OR_EARG;
    int ha[3];
    site_pos(&sy, a, ha);
    int64_t b = site_at(&sy, ha, sy.d[0][k]);
    *partner = b;
    *dE = occ[a] == occ[b] ? 0.0 : trial_dE(&sy, occ, V, a, b);
    return OR_OK;
}

/* A single trial at site a, as the sweep would run it at (seed, r, t).
 * Returns the flags (bit 0 accepted, bit 1 near-tie) or OR_EARG. */
int or_single_trial(int lattice, const int32_t L[3], int K, int S, uint8_t *occ, const double *V,
                    uint64_t seed, uint32_t replica, uint32_t sweep, int64_t a, double beta)
{
    or_sys sy;
    if (sys_init(&sy, lattice, L, K, S) != OR_OK) return OR_EARG;
    if (a < 0 || a >= sy.N) return OR_EARG;
    return do_trial(&sy, occ, V, NULL, seed, replica, sweep, a, beta, NULL, NULL);
}

/* ------------------------------------------------------------------------ */
/* Sweeps                                                                    */
/* ------------------------------------------------------------------------ */

/*
 * Run n_sweeps sweeps (global sweep indices first_sweep, ...) on one lattice.
 *
 * Partition: ncell[a] link cells along axis a with edges
 * cells[off_a + j] (off_0 = 0, off_1 = ncell[0], off_2 = ncell[0]+ncell[1]),
 * summing to L[a].  Mini-step tau = b + m*(o_x + M_x*(o_y + M_y*o_z)) with
 * M_a = the largest edge on axis a runs in ascending order; inside it the
 * cells are visited with c_x fastest, then c_y, then c_z, and a cell whose
 * edge does not exceed the offset on some axis sits the mini-step out.  The
 * active site of a cell is (cell origin + o, basis b).  Every site is active
 * exactly once per sweep.  (Sequential outer loop over i_A, inner loop over
 * i_C; Fig. 7 caption and Methods, link-cell bullet.)
 *
 * beta[j] is the inverse temperature of sweep first_sweep + j.
 * stats[0..2] += attempted, accepted, near-ties.
 * Near-ties are appended to ties (up to tie_cap, total count in *n_ties).
 * trace, when not NULL, receives every trial in execution order (needs
 * nthreads == 1; up to trace_cap entries).
 * nthreads > 1 runs the cells of one mini-step on that many OpenMP threads;
 * trials within a mini-step are independent, so the result is identical.
 */
static int run_range(int lattice, const int32_t L[3], int K, int S, const int32_t ncell[3],
                     const int32_t *cells, uint8_t *occ, const double *V, const double *W, uint64_t seed,
                     uint32_t replica, uint32_t first_sweep, int32_t n_sweeps, int32_t tau_begin,
                     int32_t tau_end, const double *beta, const or_tie *replay, int32_t n_replay,
                     int64_t *stats, or_tie *ties, int32_t tie_cap, int32_t *n_ties, or_trace *trace,
                     int64_t trace_cap, int32_t nthreads)
{
    or_sys sy;
    if (sys_init(&sy, lattice, L, K, S) != OR_OK) return OR_EARG;
    if (n_sweeps < 0 || nthreads < 1 || tau_begin < 0 || tau_end < tau_begin) return OR_EARG;
    if (trace && nthreads != 1) return OR_EARG;
    for (int64_t i = 0; i < sy.N; ++i)
        if (occ[i] >= K) return OR_EARG;
    /* symmetric V is part of the model (pair interaction) */
    for (int s = 0; s < S; ++s)
        for (int k = 0; k < K; ++k)
            for (int l = 0; l < K; ++l)
                if (V[((size_t)s * K + k) * K + l] != V[((size_t)s * K + l) * K + k]) return OR_EARG;

    /* cell origins per axis */
    int32_t *origin[3];
    int M[3];
    int off = 0;
    for (int a = 0; a < 3; ++a) {
        if (ncell[a] < 1) return OR_EARG;
        origin[a] = (int32_t *)malloc(sizeof(int32_t) * (size_t)ncell[a]);
        int acc = 0;
        M[a] = 0;
        for (int j = 0; j < ncell[a]; ++j) {
            int e = cells[off + j];
            if (e < 1) { acc = -1; break; }
            origin[a][j] = acc;
            acc += e;
            if (e > M[a]) M[a] = e;
        }
        if (acc != L[a]) {
            for (int q = 0; q <= a; ++q) free(origin[q]);
            return OR_EARG;
        }
        off += ncell[a];
    }
    const int32_t *edge[3] = {cells, cells + ncell[0], cells + ncell[0] + ncell[1]};

    or_replay rp = {replay, n_replay};
    int64_t att = 0, acc = 0, tie = 0;
    int32_t nt = 0;
    int64_t ntrace = 0;
    int m = sy.lt.m;
    int nA = M[0] * M[1] * M[2] * m;
    int64_t nC = (int64_t)ncell[0] * ncell[1] * ncell[2];

    for (int32_t js = 0; js < n_sweeps; ++js) {
        uint32_t t = first_sweep + (uint32_t)js;
        double bt = beta[js];
        int tau_hi = tau_end < nA ? tau_end : nA;
        for (int tau = tau_begin; tau < tau_hi; ++tau) {
            int b = tau % m;
            int rest = tau / m;
            int o[3];
            o[0] = rest % M[0];
            o[1] = (rest / M[0]) % M[1];
            o[2] = rest / (M[0] * M[1]);
            if (nthreads == 1) {
                for (int64_t c = 0; c < nC; ++c) {
                    int cx = (int)(c % ncell[0]);
                    int cy = (int)((c / ncell[0]) % ncell[1]);
                    int cz = (int)(c / ((int64_t)ncell[0] * ncell[1]));
                    if (o[0] >= edge[0][cx] || o[1] >= edge[1][cy] || o[2] >= edge[2][cz]) continue;
                    int64_t a = site_index(&sy, b, origin[0][cx] + o[0], origin[1][cy] + o[1],
                                           origin[2][cz] + o[2]);
                    or_trace *tr = (trace && ntrace < trace_cap) ? &trace[ntrace] : NULL;
                    int f = do_trial(&sy, occ, V, W, seed, replica, t, a, bt, &rp, tr);
                    if (trace) ++ntrace;
                    att += 1;
                    if (f & TR_ACCEPTED) acc += 1;
                    if (f & TR_TIE) {
                        tie += 1;
                        if (nt < tie_cap) {
                            ties[nt].replica = (int32_t)replica;
                            ties[nt].sweep = t;
                            ties[nt].site = a;
                            ties[nt].decision = (f & TR_ACCEPTED) ? 1 : 0;
                            ties[nt].pad = 0;
                        }
                        ++nt;
                    }
                }
            } else {
                int64_t att_l = 0, acc_l = 0, tie_l = 0;
#pragma omp parallel for num_threads(nthreads) schedule(static) reduction(+ : att_l, acc_l, tie_l)
                for (int64_t c = 0; c < nC; ++c) {
                    int cx = (int)(c % ncell[0]);
                    int cy = (int)((c / ncell[0]) % ncell[1]);
                    int cz = (int)(c / ((int64_t)ncell[0] * ncell[1]));
                    if (o[0] >= edge[0][cx] || o[1] >= edge[1][cy] || o[2] >= edge[2][cz]) continue;
                    int64_t a = site_index(&sy, b, origin[0][cx] + o[0], origin[1][cy] + o[1],
                                           origin[2][cz] + o[2]);
                    int f = do_trial(&sy, occ, V, W, seed, replica, t, a, bt, &rp, NULL);
                    att_l += 1;
                    if (f & TR_ACCEPTED) acc_l += 1;
                    if (f & TR_TIE) {
                        tie_l += 1;
#pragma omp critical(or_tie_log)
                        {
                            if (nt < tie_cap) {
                                ties[nt].replica = (int32_t)replica;
                                ties[nt].sweep = t;
                                ties[nt].site = a;
                                ties[nt].decision = (f & TR_ACCEPTED) ? 1 : 0;
                                ties[nt].pad = 0;
                            }
                            ++nt;
                        }
                    }
                }
                att += att_l;
                acc += acc_l;
                tie += tie_l;
            }
        }
    }
    for (int a = 0; a < 3; ++a) free(origin[a]);
    stats[0] += att;
    stats[1] += acc;
    stats[2] += tie;
    if (n_ties) *n_ties = nt;
    return OR_OK;
}

int or_run(int lattice, const int32_t L[3], int K, int S, const int32_t ncell[3],
           const int32_t *cells, uint8_t *occ, const double *V, uint64_t seed, uint32_t replica,
           uint32_t first_sweep, int32_t n_sweeps, const double *beta, const or_tie *replay,
           int32_t n_replay, int64_t *stats, or_tie *ties, int32_t tie_cap, int32_t *n_ties,
           or_trace *trace, int64_t trace_cap, int32_t nthreads)
{
    return run_range(lattice, L, K, S, ncell, cells, occ, V, NULL, seed, replica, first_sweep, n_sweeps, 0,
                     0x7fffffff, beta, replay, n_replay, stats, ties, tie_cap, n_ties, trace,
                     trace_cap, nthreads);
}

/* Mini-steps [tau_begin, tau_end) of the single sweep `sweep` (same
 * arguments otherwise; beta is the sweep's inverse temperature).  Running
 * consecutive ranges reproduces the full sweep. */
int or_run_ministeps(int lattice, const int32_t L[3], int K, int S, const int32_t ncell[3],
                     const int32_t *cells, uint8_t *occ, const double *V, uint64_t seed,
                     uint32_t replica, uint32_t sweep, int32_t tau_begin, int32_t tau_end, double beta,
                     const or_tie *replay, int32_t n_replay, int64_t *stats, or_tie *ties,
                     int32_t tie_cap, int32_t *n_ties, int32_t nthreads)
{
    return run_range(lattice, L, K, S, ncell, cells, occ, V, NULL, seed, replica, sweep, 1, tau_begin,
                     tau_end, &beta, replay, n_replay, stats, ties, tie_cap, n_ties, NULL, 0,
                     nthreads);
}

/* Largest |component| (half units) over the S shells' vectors. */
static int shell_reach(const or_sys *sy)
{
    int c = 0;
    for (int s = 0; s < sy->S; ++s)
        for (int n = 0; n < sy->Z[s]; ++n)
            for (int a = 0; a < 3; ++a) {
                int v = sy->d[s][n][a] < 0 ? -sy->d[s][n][a] : sy->d[s][n][a];
                if (v > c) c = v;
            }
    return c;
}

/*
 * Sweeps under the qSRO model (local energy qsro_site, V [S][K][K] and
 * W [S][K]); otherwise as or_run.  The affected set of a swap must not fold
 * onto itself through the periodic images, so every edge must exceed
 * c_max + 1 conventional cells (returns OR_EARG otherwise).  The partition
 * must satisfy the interaction-zone rule 2 l > 2 + 2 c_max (or_lmin with
 * liz = 1) for its mini-steps to be independent; that is the caller's.
 */
int or_run_qsro(int lattice, const int32_t L[3], int K, int S, const int32_t ncell[3], const int32_t *cells,
                uint8_t *occ, const double *V, const double *W, uint64_t seed, uint32_t replica,
                uint32_t first_sweep, int32_t n_sweeps, const double *beta, const or_tie *replay, int32_t n_replay,
                int64_t *stats, or_tie *ties, int32_t tie_cap, int32_t *n_ties, int32_t nthreads)
{
    or_sys sy;
    if (!W || sys_init(&sy, lattice, L, K, S) != OR_OK) return OR_EARG;
    int c = shell_reach(&sy);
    for (int a = 0; a < 3; ++a)
        if (L[a] <= c + 1) return OR_EARG;
    return run_range(lattice, L, K, S, ncell, cells, occ, V, W, seed, replica, first_sweep, n_sweeps, 0, 0x7fffffff,
                     beta, replay, n_replay, stats, ties, tie_cap, n_ties, NULL, 0, nthreads);
}

/* qSRO local energies of every site (for the pins), and the qSRO energy
 * change of one swap of site a with its partner in direction k (occ is left
 * unchanged; *b_out receives the partner). */
int or_qsro_local_energy(int lattice, const int32_t L[3], int K, int S, const uint8_t *occ, const double *V,
                         const double *W, double *e)
{
    or_sys sy;
    if (sys_init(&sy, lattice, L, K, S) != OR_OK) return OR_EARG;
    for (int64_t i = 0; i < sy.N; ++i)
        if (occ[i] >= K) return OR_EARG;
    for (int64_t i = 0; i < sy.N; ++i) e[i] = qsro_site(&sy, occ, V, W, i);
    return OR_OK;
}

int or_qsro_delta_e(int lattice, const int32_t L[3], int K, int S, uint8_t *occ, const double *V, const double *W,
                    int64_t a, int32_t k, double *dE, int64_t *b_out)
{
    or_sys sy;
    if (sys_init(&sy, lattice, L, K, S) != OR_OK) return OR_EARG;
    if (a < 0 || a >= sy.N || k < 0 || k >= sy.Z[0]) return OR_EARG;
    int c = shell_reach(&sy);
    for (int ax = 0; ax < 3; ++ax)
        if (L[ax] <= c + 1) return OR_EARG;
    int ha[3];
    site_pos(&sy, a, ha);
    int64_t b = site_at(&sy, ha, sy.d[0][k]);
    *b_out = b;
    *dE = occ[a] == occ[b] ? 0.0 : qsro_dE(&sy, occ, V, W, a, b, k);
    return OR_OK;
}

/* Number of OpenMP threads available to the timing variant (1 without
 * OpenMP). */
int or_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Replica exchange between temperature slots                                */
/* ------------------------------------------------------------------------ */

/*
 * One round of replica exchange (parallel tempering: Swendsen and Wang, PRL
 * 57 (1986) 2607; Geyer 1991; Hukushima and Nemoto, JPSJ 65 (1996) 1604) over
 * R replicas of one lattice held in R temperature slots.  The paper runs its
 * temperatures as independent chains (Supplementary, parallelization
 * opportunities); exchanging configurations between neighbouring
 * temperatures is the textbook extension of such a ladder.
 *
 * rep_at[i] is the replica held by slot i (inverse temperature
 * beta_slot[i]); E[r] is the energy of replica r.  Round j pairs slots
 * (i, i + 1) for i = j mod 2, j mod 2 + 2, ... while i + 1 < R.  With
 * a = rep_at[i], b = rep_at[i + 1], the joint weight of the two slots changes
 * by exp(x), x = (beta_slot[i] - beta_slot[i + 1]) * (E[a] - E[b]), when they
 * trade replicas, so the trade is accepted when x >= 0 and otherwise when
 * u < exp(x), u the 53-bit uniform of Philox4x32-10 on counter
 * (i, 0, j, 0xffffffff) under the run's key (no trial uses replica index
 * 0xffffffff).  |u - exp(x)| < 1e-12 is a near-tie: it is logged as
 * {replica -1, sweep j, site i, decision}, and a replay entry with those
 * keys overrides the decision.  Accepted pairs swap rep_at[i] and
 * rep_at[i + 1].  stats[2 i] counts the attempts of pair i, stats[2 i + 1]
 * its acceptances.  Returns OR_EARG if rep_at holds an index outside [0, R).
 */
int or_exchange(int R, const double *E, const double *beta_slot, int32_t *rep_at, uint64_t seed,
                uint32_t round, const or_tie *replay, int32_t n_replay, int64_t *stats, or_tie *ties,
                int32_t tie_cap, int32_t *n_ties)
{
    for (int i = 0; i < R; ++i)
        if (rep_at[i] < 0 || rep_at[i] >= R) return OR_EARG;
    or_replay rp = {replay, n_replay};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int i = (int)(round & 1u); i + 1 < R; i += 2) {
        int a = rep_at[i], b = rep_at[i + 1];
        double x = (beta_slot[i] - beta_slot[i + 1]) * (E[a] - E[b]);
        int accept;
        if (x >= 0.0) {
            accept = 1;
        } else {
            uint32_t ctr[4] = {(uint32_t)i, 0u, round, 0xffffffffu};
            uint32_t w[4];
            or_philox4x32_10(ctr, key, w);
            double P = exp(x);
            double u = u53(w);
            accept = u < P;
            if (fabs(u - P) < 1e-12) {
                int dec;
                if (replay_lookup(&rp, -1, round, i, &dec)) accept = dec;
                if (*n_ties < tie_cap) {
                    or_tie *e = &ties[*n_ties];
                    e->replica = -1;
                    e->sweep = round;
                    e->site = i;
                    e->decision = accept;
                    e->pad = 0;
                }
                *n_ties += 1;
            }
        }
        stats[2 * i] += 1;
        if (accept) {
            stats[2 * i + 1] += 1;
            rep_at[i] = b;
            rep_at[i + 1] = a;
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Heat capacity from energy fluctuations                                    */
/* ------------------------------------------------------------------------ */

/*
 * Heat capacity per site, in units of k_B, from n energies recorded at one
 * inverse temperature beta: c = beta^2 (<E^2> - <E>^2) / N (the fluctuation
 * formula of the canonical ensemble; the paper reads its specific-heat peaks
 * off annealing runs, Results on the phase transitions and Methods on the
 * annealing protocol).  Two passes in binary64, j ascending:
 * m = (sum E_j) / n, v = (sum (E_j - m)^2) / n, c = (beta beta) v / N.
 */
double or_heat_capacity(int n, const double *E, double beta, int64_t N)
{
    double m = 0.0;
    for (int j = 0; j < n; ++j) m = m + E[j];
    m = m / (double)n;
    double v = 0.0;
    for (int j = 0; j < n; ++j) {
        double d = E[j] - m;
        v = v + d * d;
    }
    v = v / (double)n;
    return beta * beta * v / (double)N;
}

/* ------------------------------------------------------------------------ */
/* Local energies and clusters                                               */
/* ------------------------------------------------------------------------ */

/*
 * Local energy of every site, e_i = 1/2 sum_s sum_t n_i[s][t] V_s[sigma_i][t]
 * with n_i[s][t] the number of shell-s neighbours of i with species t
 * (periodic images counted with multiplicity), accumulated s, t ascending in
 * binary64.  The half makes the local energies add up to E (Eq. Linear_EPI
 * gives the per-site form; the paper computes local energies to find its
 * nanostructures, Methods after Tab. 4).
 */
static double local_energy_site(const or_sys *sy, const uint8_t *occ, const double *V, int64_t i)
{
    int K = sy->K, S = sy->S;
    int h[3];
    site_pos(sy, i, h);
    int n[OR_MAXS][OR_MAXK];
    memset(n, 0, sizeof(n));
    for (int s = 0; s < S; ++s)
        for (int k = 0; k < sy->Z[s]; ++k) n[s][occ[site_at(sy, h, sy->d[s][k])]] += 1;
    double acc = 0.0;
    for (int s = 0; s < S; ++s)
        for (int t = 0; t < K; ++t) acc = acc + (double)n[s][t] * V[((size_t)s * K + occ[i]) * K + t];
    return acc * 0.5;
}

int or_local_energy(int lattice, const int32_t L[3], int K, int S, const uint8_t *occ, const double *V,
                    double *e)
{
    or_sys sy;
    if (sys_init(&sy, lattice, L, K, S) != OR_OK) return OR_EARG;
    for (int64_t i = 0; i < sy.N; ++i)
        if (occ[i] >= K) return OR_EARG;
    for (int64_t i = 0; i < sy.N; ++i) e[i] = local_energy_site(&sy, occ, V, i);
    return OR_OK;
}

/* The same for the n listed sites only (e[j] for site idx[j]); occupancy
 * values are not checked. */
int or_local_energy_at(int lattice, const int32_t L[3], int K, int S, const uint8_t *occ, const double *V,
                       const int64_t *idx, int64_t n, double *e)
{
    or_sys sy;
    if (sys_init(&sy, lattice, L, K, S) != OR_OK) return OR_EARG;
    for (int64_t j = 0; j < n; ++j) {
        if (idx[j] < 0 || idx[j] >= sy.N) return OR_EARG;
        e[j] = local_energy_site(&sy, occ, V, idx[j]);
    }
    return OR_OK;
}

/*
 * Clusters of low-energy sites (the paper's union-find step, Methods after
 * Tab. 4): site i is marked when e[i] <= threshold; marked nearest neighbours
 * (shell 1, periodic) belong to the same cluster.  label[i] is the smallest
 * site index of i's cluster, or -1 for an unmarked site; size[i] is the
 * number of sites of the cluster whose smallest index is i, else 0.  Found by
 * a flood fill from each unlabelled marked site in index order (the first
 * site reached is the smallest of its cluster).  *n_clusters counts them.
 * `stack` is caller scratch of N entries.
 */
int or_clusters(int lattice, const int32_t L[3], const double *e, double threshold, int32_t *label, int32_t *size,
                int64_t *n_clusters, int64_t *stack)
{
    or_sys sy;
    if (sys_init(&sy, lattice, L, 2, 1) != OR_OK) return OR_EARG;
    if (sy.N > 0x7fffffffLL) return OR_EARG;
    for (int64_t i = 0; i < sy.N; ++i) {
        label[i] = -1;
        size[i] = 0;
    }
    int64_t nc = 0;
    for (int64_t i = 0; i < sy.N; ++i) {
        if (!(e[i] <= threshold) || label[i] >= 0) continue;
        int64_t top = 0;
        stack[top++] = i;
        label[i] = (int32_t)i;
        int32_t count = 0;
        while (top > 0) {
            int64_t a = stack[--top];
            ++count;
            int h[3];
            site_pos(&sy, a, h);
            for (int k = 0; k < sy.Z[0]; ++k) {
                int64_t j = site_at(&sy, h, sy.d[0][k]);
                if (e[j] <= threshold && label[j] < 0) {
                    label[j] = (int32_t)i;
                    stack[top++] = j;
                }
            }
        }
        size[i] = count;
        ++nc;
    }
    *n_clusters = nc;
    return OR_OK;
}
