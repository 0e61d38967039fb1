/*
 * smcx.h -- C ABI of libsmcx, link-cell parallel canonical swap Metropolis
 * Monte Carlo with a multi-shell effective pair interaction (EPI) energy on
 * BCC / FCC lattices, for AMD Instinct MI355X (gfx950).
 *
 * Method (paper: "Revealing Nanostructures in High-Entropy Alloys via
 * Machine-Learning Accelerated Scalable Monte Carlo Simulation"):
 *   - a sweep is n_A sequential mini-steps; a mini-step makes one trial in
 *     every link cell, all of them independent (Results, "Performance of the
 *     SMC-X algorithm", Fig. 1a/1c; Methods, "Implementation of SMC-GPU",
 *     link-cell bullet; Fig. 7 caption);
 *   - a trial swaps the species of a site with one of its nearest
 *     neighbours and is accepted with probability min(1, exp(-beta dE))
 *     (Supplementary, "Monte Carlo Simulation Algorithms");
 *   - E = 1/2 sum_i sum_s sum_{d in D_s} V_s[sigma_i][sigma_{i+d}] (Methods,
 *     "The EPI and qSRO model", Eq. Linear_EPI and Eq. Total_EPI), and dE of
 *     a swap is twice the change of the two local energies (same section).
 *
 * Conventions fixed by this library (the paper leaves them open):
 *   - positions in half lattice constants; BCC basis (0,0,0),(1,1,1); FCC
 *     basis (0,0,0),(1,1,0),(1,0,1),(0,1,1); periodic boundaries;
 *   - site index i = b + m*(x + Lx*(y + Ly*z)) for basis b (m = 2 BCC, 4 FCC)
 *     and conventional cell (x, y, z); one uint8 species per site;
 *   - shells D_s: lattice vectors of the s-th smallest length, sorted
 *     lexicographically; D_1 fixes the partner direction k;
 *   - per-axis partition into link cells; mini-step
 *     tau = b + m*(o_x + M_x*(o_y + M_y*o_z)) ascending, M_a the largest cell
 *     edge on axis a; a cell whose edge does not exceed an offset sits that
 *     mini-step out;
 *   - random numbers: Philox4x32-10 (Salmon et al., SC'11), key = seed,
 *     counter = (site_lo, site_hi, sweep, replica); partner
 *     k = floor(w0 * Z_1 / 2^32); u = ((w1 << 21) | (w2 >> 11)) * 2^-53;
 *   - dE = sum_s sum_t (n_a - n_b)[s][t] * (V_s[q][t] - V_s[p][t]) in binary64,
 *     s then t ascending, no fused multiply-add, where n_a counts the
 *     neighbours of the active site a (species p) excluding the partner b
 *     (species q) and n_b those of b excluding a; trials with p == q are
 *     attempted but not accepted; accept if dE <= 0, else if u < exp(-beta dE);
 *     |u - exp(-beta dE)| < 1e-12 is a near-tie and is logged.
 *
 * Memory and threading: the caller allocates every large device buffer
 * (occupancy, workspace, counts, statistics, tie logs) and keeps it alive
 * while the handle uses it.  The library never allocates device memory.
 * Calls taking a stream are asynchronous on it unless they return host
 * values, in which case they synchronise that stream before returning.
 * A handle must not be used from two threads at once.  No C++ exception
 * crosses this interface; every call returns an SMCX_* status.
 */
#ifndef SMCX_H
#define SMCX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SMCX_VERSION 100

/* status codes */
#define SMCX_OK 0
#define SMCX_E_INVALID_ARG (-1)   /* bad argument; smcx_last_error() says which */
#define SMCX_E_UNSUPPORTED (-2)   /* valid request the library cannot serve */
#define SMCX_E_NOT_READY (-3)     /* set_epi not called yet */
#define SMCX_E_HIP (-4)           /* a HIP runtime call failed */
#define SMCX_E_WORKSPACE (-5)     /* workspace too small */

/* lattice kinds */
#define SMCX_BCC 0
#define SMCX_FCC 1

/* sweep execution modes (all give the same trajectory) */
#define SMCX_MODE_AUTO 0        /* persistent for lattices of at most 65536 sites, else stream where
                                   row windows apply or R == 1, else persistent */
#define SMCX_MODE_STREAM 1      /* one launch per mini-step, batched over replicas */
#define SMCX_MODE_PERSISTENT 2  /* one launch for all sweeps, one workgroup per replica */
#define SMCX_MODE_PLAIN 3       /* one launch per replica per mini-step (baseline loop) */

typedef struct smcx_lattice smcx_lattice;

/* Near-tie record (24 bytes): the trial of `site` in `sweep` of `replica`
 * came within 1e-12 of its acceptance threshold; `decision` is 1 when it was
 * accepted. */
typedef struct {
    int32_t replica;
    uint32_t sweep;
    int64_t site;
    int32_t decision;
    int32_t pad;
} smcx_tie;

/* Problem description.  All pointers are host pointers, read during
 * smcx_lattice_init only. */
typedef struct {
    int32_t lattice;       /* SMCX_BCC or SMCX_FCC */
    int32_t n_species;     /* K, 2 .. 8 */
    int32_t n_shells;      /* S, 1 .. 4 */
    int32_t n_replicas;    /* R >= 1; replicas are stored back to back in occ */
    const int32_t *dims;   /* [R][3] conventional cells per axis, each >= 2 */
    const int32_t *ell;    /* [R] link-cell edge for the default partition rule
                              (n = max(1, L / ell) cells per axis, edges L / n or
                              L / n + 1, larger first), or NULL for 4.  Values
                              below the minimum edge are raised to it. */
    const int32_t *ncell;  /* [R][3] explicit partition: cells per axis, or NULL */
    const int32_t *cells;  /* explicit partition: for each replica, the edges of
                              the x cells, then y, then z, concatenated; each
                              axis sums to its dimension and every edge is at
                              least the minimum unless the axis has one cell */
    int32_t tile[3];       /* link cells per workgroup tile along x, y, z
                              (product <= 256), or {0,0,0} for the default
                              (16,4,2) */
    uint32_t flags;        /* SMCX_FLAG_* bits */
} smcx_desc;

/* desc.flags: give each workgroup two tile windows, so that the next tile's
 * window streams into LDS while the current tile's trials run (the default
 * stages one window at a time, with half the LDS per workgroup and so more
 * workgroups per CU; both give the same trajectory). */
#define SMCX_FLAG_DOUBLE_BUFFER 1u

/* desc.flags: in stream mode, stage tiles of link cells for every mini-step
 * even where whole x-rows would fit.  By default, when every cell edge leaves
 * room for consecutive offsets to share a window (2*edge > 3 + c_max), all
 * replicas split the same way and a row of link cells fits one workgroup,
 * stream mode gives each workgroup whole x-rows and runs all mini-steps with
 * the same (o_y, o_z) in one launch.  Both give the same trajectory. */
#define SMCX_FLAG_TILES 2u

int smcx_version(void);

/* Thread-local text of the last error (empty string when none). */
const char *smcx_last_error(void);

/* Smallest link-cell edge (conventional cells) for which the trials of one
 * mini-step are independent: 2*ell > 2 + c_max, c_max the largest |component|
 * (half-lattice units) over the first n_shells shells.  Returns the edge, or
 * a negative status. */
int smcx_min_cell_edge(int32_t lattice, int32_t n_shells);

/* Device workspace (bytes) that smcx_lattice_init needs for this
 * description.  It holds the per-replica metadata and tables and a padded
 * working copy of the occupancy with a 2-cell periodic halo. */
int smcx_workspace_size(const smcx_desc *desc, size_t *bytes);

/* Create a handle for R replicas of one lattice kind: the configuration
 * (one species per site), the coordination shells of the energy model and
 * the partition of each replica into link cells whose trials of one
 * mini-step are independent (Methods, "Implementation of SMC-GPU", link-cell
 * bullet; Fig. 7; Results, "Performance of the SMC-X algorithm", the
 * LIZ / LIZ+ argument).
 *   occ_dev  device uint8 [sum_r N_r], replicas back to back in site-index
 *            order; every value must be < K.  Caller-owned; the sweeps
 *            mutate it in place.
 *   ws_dev   device workspace of ws_bytes >= smcx_workspace_size, 256-byte
 *            aligned, caller-owned.
 * Uploads the tables on `stream`, checks on the device that every species
 * is < K, and synchronises.  The handle keeps both pointers; their memory
 * must outlive it.  Errors: SMCX_E_INVALID_ARG (bad description, a species
 * >= K, a partition below the minimum edge, misaligned or NULL pointers),
 * SMCX_E_WORKSPACE (ws_bytes too small), SMCX_E_HIP. */
int smcx_lattice_init(smcx_lattice **out, const smcx_desc *desc, uint8_t *occ_dev, void *ws_dev,
                      size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * handle as smcx_lattice_init, with the workspace taken from a static array
 * inside the library instead of a caller buffer.  Each device the library
 * runs on holds its own array of 64 MiB (SMCX_STATIC_WORKSPACE_BYTES) until
 * the process ends; descriptions whose smcx_workspace_size exceeds it are
 * rejected with SMCX_E_WORKSPACE.  Nothing is allocated: the tables are
 * uploaded with asynchronous copies on `stream`, which is synchronised.
 * occ_dev as for smcx_lattice_init (caller-owned, every value < K).
 * Every handle made by this call on one device shares that device's array:
 * a later call on the device takes it over, after which the earlier handle's
 * calls fail with SMCX_E_INVALID_ARG (destroy it as usual), and calls through
 * such handles that overlap in time on one device race.  Errors: as for
 * smcx_lattice_init, SMCX_E_WORKSPACE when the description does not fit. */
#define SMCX_STATIC_WORKSPACE_BYTES (64u << 20)
int smcx_lattice_init_static(smcx_lattice **out, const smcx_desc *desc, uint8_t *occ_dev, void *stream);

int smcx_lattice_destroy(smcx_lattice *h);

/* Partition actually used by replica r: ncell_out[3] cells per axis and the
 * edges (x cells, then y, then z) in cells_out, which must hold
 * Lx + Ly + Lz entries (host memory, caller-owned); *n_ministeps =
 * M_x*M_y*M_z*m, the n_A sequential mini-steps of a sweep (Fig. 7 caption:
 * the outer loop over the site index within a link cell is sequential, the
 * inner loop over link cells parallel; Tab. 4 for link cells of 3 and 4).
 * Feed these to a replay of the same trajectory.  Errors:
 * SMCX_E_INVALID_ARG (NULL pointers, replica out of range). */
int smcx_get_schedule(const smcx_lattice *h, int32_t replica, int32_t *ncell_out,
                      int32_t *cells_out, int32_t *n_ministeps);

/* Set the EPI tensor V (host, binary64, [S][K][K], eV; copied): the pair
 * interaction of species k and l at shell distance s (Methods, "The EPI and
 * qSRO model", Eq. Linear_EPI and Eq. Total_EPI, with the energy written as
 * E = 1/2 sum_i sum_s sum_{d in D_s} V_s[sigma_i][sigma_{i+d}]).  V must be
 * symmetric in (k, l) exactly.  Tables D[s][t][p][q] = V_s[q][t] - V_s[p][t]
 * are uploaded on `stream`, which is synchronised.  Errors:
 * SMCX_E_INVALID_ARG (NULL, asymmetric or non-finite V), SMCX_E_HIP. */
int smcx_set_epi(smcx_lattice *h, const double *V, void *stream);

/*
 * Run n_sweeps sweeps on every replica, global sweep indices first_sweep ..
 * first_sweep + n_sweeps - 1, mutating occ_dev in place.  A sweep is the n_A
 * mini-steps in order, a mini-step one swap trial in every link cell
 * (Methods, "Implementation of SMC-GPU", link-cell and random-number
 * bullets; Fig. 7); a trial swaps a site with a random nearest neighbour and
 * is accepted with probability min(1, exp(-beta dE)) (Supplementary, "Monte
 * Carlo Simulation Algorithms", the acceptance equation), dE being twice
 * the change of the two local energies (Methods, "The EPI and qSRO model").
 *   beta_dev   device double [n_sweeps][R] inverse temperatures (1/eV)
 *   stats_dev  device int64 [R][3], incremented by attempted, accepted and
 *              near-tie counts
 *   ties_dev   device smcx_tie [tie_cap] (may be NULL when tie_cap == 0)
 *   tie_count_dev device int32 [1]: incremented once per near-tie; entries
 *              past tie_cap are counted but not stored
 *   mode       SMCX_MODE_*
 * All pointers are device memory owned by the caller.  Asynchronous on
 * `stream`.  Errors: SMCX_E_INVALID_ARG (negative n_sweeps, missing buffers,
 * bad mode), SMCX_E_NOT_READY before smcx_set_epi, SMCX_E_HIP.
 */
int smcx_sweep(smcx_lattice *h, int32_t n_sweeps, uint64_t seed, uint32_t first_sweep,
               const double *beta_dev, int64_t *stats_dev, smcx_tie *ties_dev, int32_t tie_cap,
               int32_t *tie_count_dev, int32_t mode, void *stream);

/*
 * Run only mini-steps [tau_begin, tau_end) of global sweep `sweep` (beta_dev:
 * device double [R], the sweep's inverse temperatures; the other arguments as
 * for smcx_sweep).  Replicas with fewer mini-steps run those they have.  A
 * full sweep is tau_begin = 0, tau_end = the largest n_ministeps; splitting a
 * sweep into ranges gives the same trajectory.  Used to checkpoint inside a
 * sweep and to check single mini-steps against a sequential replay.
 */
int smcx_sweep_partial(smcx_lattice *h, uint32_t sweep, int32_t tau_begin, int32_t tau_end,
                       uint64_t seed, const double *beta_dev, int64_t *stats_dev,
                       smcx_tie *ties_dev, int32_t tie_cap, int32_t *tie_count_dev, int32_t mode,
                       void *stream);

/* Directed pair counts C[r][s][k][l] = #{(i, d in D_s) : sigma_i = k,
 * sigma_{i+d} = l} of every replica into counts_dev (device int64
 * [R][S][K][K], overwritten).  These are the per-shell pair numbers of the
 * EPI features (Methods, "The EPI and qSRO model").  Asynchronous. */
int smcx_pair_counts(smcx_lattice *h, int64_t *counts_dev, void *stream);

/* Energies E[r] = 1/2 sum_{s,k,l} C[r][s][k][l] V_s[k][l] (binary64, s, k, l
 * ascending) into E_host [R]; counts_dev as for smcx_pair_counts.
 * Synchronises the stream.  (Eq. Total_EPI.) */
int smcx_energy(smcx_lattice *h, int64_t *counts_dev, double *E_host, void *stream);

/* Warren-Cowley short-range order alpha[r][s][k][l] =
 * 1 - C N / (Z_s N_k N_l) into alpha_host [R][S][K][K] (host double,
 * caller-owned), from the directed pair counts (recomputed into counts_dev
 * as for smcx_pair_counts).  The textbook parameter (Cowley 1950) over the
 * per-shell pair numbers that the paper's pair fractions pi_m^{pp'} are built
 * from (Methods, "The EPI and qSRO model").  Returns SMCX_E_INVALID_ARG when
 * a species is absent from a replica.  Synchronises the stream. */
int smcx_sro(smcx_lattice *h, int64_t *counts_dev, double *alpha_host, void *stream);

/* Energies as smcx_energy, left on the device: counts_dev [R][S][K][K] int64
 * is overwritten with the pair counts, E_dev [R] binary64 receives
 * E[r] = 1/2 sum_{s,k,l} C V (s, k, l ascending, the same rounding as
 * smcx_energy).  Asynchronous on `stream`, no host synchronisation (so it
 * can be recorded in a graph).  (Eq. Total_EPI.) */
int smcx_energy_dev(smcx_lattice *h, int64_t *counts_dev, double *E_dev, void *stream);

/* One round of replica exchange (parallel tempering) between R temperature
 * slots, for replicas of one size.  Not part of the paper, whose
 * temperatures run as independent chains (Supplementary, parallelization
 * opportunities); the rule is the textbook one (Swendsen and Wang 1986;
 * Hukushima and Nemoto 1996).
 *   beta_slot_dev [R] binary64: inverse temperature of slot i (any order).
 *   rep_at_dev [R] int32, in/out: the replica held by slot i, a permutation
 *     of 0 .. R-1 (start from the identity).  Entries outside [0, R) leave
 *     their pair, and their replica's beta, untouched.
 *   Round `round` computes every replica's energy (counts_dev, E_dev as for
 *   smcx_energy_dev) and visits the slot pairs (i, i + 1), i = round mod 2,
 *   round mod 2 + 2, ...: with a = rep_at[i], b = rep_at[i + 1] and
 *   x = (beta_slot[i] - beta_slot[i + 1]) (E[a] - E[b]) the slots trade their
 *   replicas when x >= 0, else when u < exp(x), u the 53-bit uniform of
 *   Philox4x32-10 with key `seed` on counter (i, 0, round, 0xffffffff) (no
 *   trial uses replica index 0xffffffff).  |u - exp(x)| < 1e-12 is a
 *   near-tie, appended to ties_dev as {replica -1, sweep round, site i,
 *   decision} (tie_count_dev counts past tie_cap as for smcx_sweep).
 *   xstats_dev [R-1][2] int64, accumulated: attempts and trades of pair i.
 *   beta_dev [n_beta_rows][R] binary64, written: every row gets each
 *     replica's new inverse temperature, ready as the beta argument of the
 *     next smcx_sweep of n_beta_rows sweeps (n_beta_rows may be 0).
 * All pointers are device memory owned by the caller.  Asynchronous, no
 * host synchronisation, no allocation.  Errors: SMCX_E_INVALID_ARG for
 * missing buffers, round < 0 or replicas of different sizes;
 * SMCX_E_NOT_READY before smcx_set_epi. */
int smcx_exchange(smcx_lattice *h, int32_t round, uint64_t seed, const double *beta_slot_dev,
                  int32_t *rep_at_dev, double *beta_dev, int32_t n_beta_rows, int64_t *counts_dev,
                  double *E_dev, int64_t *xstats_dev, smcx_tie *ties_dev, int32_t tie_cap,
                  int32_t *tie_count_dev, void *stream);

/* qSRO model (Methods, "The EPI and qSRO model", Eq. quadratic_local_SRO):
 * the local energy of a site with species p is
 *   E_i = sum_m sum_t V_m[p][t] (n_i[m][t] / Z_m) + sum_m W_m[p] (n_i[m][p] / Z_m)^2
 * (pair fractions of the centre-neighbour pairs of shell m; m, then t,
 * ascending, binary64).  V [S][K][K] (symmetric) and W [S][K] are host
 * arrays, copied.  Synchronises the stream.  Errors: SMCX_E_INVALID_ARG
 * (NULL, asymmetric or non-finite V, non-finite W). */
int smcx_set_qsro(smcx_lattice *h, const double *V, const double *W, void *stream);

/* n_sweeps sweeps of every replica under the qSRO model, in the same
 * mini-step order and with the same per-trial random numbers, partner and
 * acceptance rule (near-tie log included) as smcx_sweep.  A swap changes the
 * local energy of every site that has a or b in one of its shells, so its
 * energy change is the sum of E_after - E_before over that affected set:
 * a, b and every shell neighbour of either, without duplicates, in
 * lexicographic order of the half-unit displacement from a (the paper's rule
 * for models beyond pairs: add up the local energies of the interaction
 * zone).  A wave takes one trial and its lanes the affected sites
 * (sub-move parallelism).
 *   beta_host [n_sweeps][R] binary64 (host).
 *   stats_dev, ties_dev, tie_cap, tie_count_dev: as for smcx_sweep.
 * Requirements: every link-cell edge (on axes of more than one cell) at
 * least the interaction-zone minimum, the smallest l with 2 l > 2 + 2 c_max
 * (c_max: largest shell-vector component in half units; 4 for BCC or FCC
 * with 2 shells, 5 for BCC with 4), so that a mini-step's trials do not
 * see each other's swaps; every edge above c_max + 1; fewer than 2^31 sites
 * per replica.  Asynchronous.  Errors: SMCX_E_INVALID_ARG,
 * SMCX_E_UNSUPPORTED, SMCX_E_NOT_READY before smcx_set_qsro. */
int smcx_sweep_qsro(smcx_lattice *h, int32_t n_sweeps, uint64_t seed, uint32_t first_sweep,
                    const double *beta_host, int64_t *stats_dev, smcx_tie *ties_dev, int32_t tie_cap,
                    int32_t *tie_count_dev, void *stream);

/* Local energy of every site of one replica: e_dev [N_r] binary64 receives
 * e_i = 1/2 sum_s sum_t n_i[s][t] V_s[sigma_i][t] (n_i[s][t]: shell-s
 * neighbours of species t, periodic images with multiplicity; s, t
 * ascending), so that sum_i e_i = E.  The per-site form of Eq. Linear_EPI;
 * the paper computes it to find nanostructures (Methods after Tab. 4).
 * Asynchronous.  Errors: SMCX_E_INVALID_ARG (replica out of range, NULL),
 * SMCX_E_UNSUPPORTED for N_r >= 2^31, SMCX_E_NOT_READY before smcx_set_epi. */
int smcx_local_energy(smcx_lattice *h, int32_t replica, double *e_dev, void *stream);

/* Clusters of low-energy sites (the paper's union-find step, Methods after
 * Tab. 4): site i of the replica is marked when e_dev[i] <= threshold, and
 * marked nearest neighbours (shell 1, periodic) join one cluster.
 *   label_dev [N_r] int32, written: the smallest site index of i's cluster,
 *     or -1 for an unmarked site (unique, whatever the order of unions).
 *   size_dev [N_r] int32, written: the number of sites of the cluster whose
 *     smallest site is i, else 0.
 *   n_clusters_dev [1] int64, written: the number of clusters.
 * Device memory owned by the caller; asynchronous, no allocation.  Errors:
 * SMCX_E_INVALID_ARG (replica out of range, NULL), SMCX_E_UNSUPPORTED for
 * N_r >= 2^31. */
int smcx_clusters(smcx_lattice *h, int32_t replica, const double *e_dev, double threshold,
                  int32_t *label_dev, int32_t *size_dev, int64_t *n_clusters_dev, void *stream);

/* Stepwise anneal with energy recording (the paper's protocol: start hot,
 * lower T in steps, discard sweeps at each temperature before measuring;
 * Methods, MC simulation paragraph after Tab. 4).  Step s = 0 .. n_steps-1
 * runs `warmup` sweeps, then `record` sweeps each followed by the energies
 * of every replica, all at beta_steps_dev[s][r]; sweep indices run from
 * first_sweep on, (warmup + record) per step.
 *   beta_steps_dev [n_steps][R] binary64 (device).
 *   counts_dev [R][S][K][K] int64: scratch, overwritten.
 *   E_dev [n_steps][record][R] binary64: recorded energies (smcx_energy_dev).
 *   cv_dev [n_steps][R] binary64: heat capacity per site in units of k_B,
 *     beta^2 Var(E) / N_r over the step's recorded energies (two passes,
 *     j ascending: m = sum E / n, v = sum (E - m)^2 / n, c = beta beta v / N).
 *   stats_dev, ties_dev, tie_cap, tie_count_dev, mode: as for smcx_sweep.
 * counts_dev, E_dev and cv_dev may be NULL when record == 0.  Everything is
 * enqueued on `stream` without host synchronisation.  Errors:
 * SMCX_E_INVALID_ARG (negative sizes, missing buffers, sweep index past
 * 2^32), SMCX_E_NOT_READY before smcx_set_epi. */
int smcx_anneal(smcx_lattice *h, int32_t n_steps, int32_t warmup, int32_t record, uint64_t seed,
                uint32_t first_sweep, const double *beta_steps_dev, int64_t *counts_dev, double *E_dev,
                double *cv_dev, int64_t *stats_dev, smcx_tie *ties_dev, int32_t tie_cap,
                int32_t *tie_count_dev, int32_t mode, void *stream);

/* Backward of the energy with respect to the EPI: stateless batched pair
 * counts for B configurations of one geometry.  E_b = 1/2 <C_b, V> is linear
 * in V, so dE_b/dV = C_b / 2; the paper fits its EPI by Adam and
 * back-propagation on these features (Methods, "The EPI and qSRO model",
 * Eq. Total_EPI and the fitting paragraph).
 *   dims          host int32 [3], conventional cells per axis (each >= 2)
 *   occ_batch_dev device uint8 [B][N] (N = m * dims[0]*dims[1]*dims[2]),
 *                 every value < n_species (checked on the device)
 *   counts_dev    device int64 [B][S][K][K] (overwritten)
 * Device memory owned by the caller.  Asynchronous, except that a species
 * check failure is reported: the call synchronises `stream` to read the
 * check's flag.  Errors: SMCX_E_INVALID_ARG (bad lattice, K, S, dims, B,
 * NULL pointers, a lattice so small that a site is its own neighbour, a
 * species >= n_species), SMCX_E_HIP. */
int smcx_energy_backward(int32_t lattice, const int32_t *dims, int32_t n_species,
                         int32_t n_shells, const uint8_t *occ_batch_dev, int32_t B,
                         int64_t *counts_dev, void *stream);

/* Energies of B configurations from their pair counts (the forward of the
 * EPI fit; Methods, "The EPI and qSRO model", Eq. Total_EPI: the energy is
 * linear in the pair numbers):
 *   E_dev[b] = 1/2 sum_i counts_dev[b][i] V_dev[i], i ascending, binary64
 * (the rounding of smcx_energy), with n_terms = S*K*K entries per
 * configuration.  counts_dev device int64 [B][n_terms] (from
 * smcx_energy_backward), V_dev device double [n_terms], E_dev device double
 * [B]; caller-owned.  Asynchronous.  Errors: SMCX_E_INVALID_ARG (B < 0,
 * n_terms < 1, NULL pointers), SMCX_E_HIP. */
int smcx_energy_of_counts(const int64_t *counts_dev, const double *V_dev, int32_t B, int32_t n_terms,
                          double *E_dev, void *stream);

/* Gradient of sum_b g[b] E_b with respect to V for E_b = 1/2 <C_b, V> (the
 * back-propagation step of the EPI fit; Methods, "The EPI and qSRO model"):
 *   grad_dev[i] = 1/2 sum_b g_dev[b] counts_dev[b][i], b ascending, binary64.
 * counts_dev device int64 [B][n_terms], g_dev device double [B], grad_dev
 * device double [n_terms] (overwritten; zero when B == 0); caller-owned.
 * Asynchronous.  Errors: SMCX_E_INVALID_ARG, SMCX_E_HIP. */
int smcx_energy_grad(const int64_t *counts_dev, const double *g_dev, int32_t B, int32_t n_terms, double *grad_dev,
                     void *stream);

/*
 * Temperature ladder as a replayable graph (temperatures are independent
 * chains, the paper's temperature parallelism: Supplementary, "Parallelization
 * opportunities in Monte Carlo simulation"; Methods after Tab. 4, the two GPUs
 * used by temperature parallelization).  Captures, on `stream`, one
 * persistent launch that runs n_sweeps sweeps on every replica with the
 * fixed inverse temperatures beta_dev [R] (device double).  The first sweep
 * index is read from *sweep_counter_dev (device uint32) when the graph runs
 * and advanced by n_sweeps at its end, so every replay continues the chain.
 * *graph_out receives an executable graph for smcx_graph_launch.  `stream`
 * must be a created stream (the legacy default stream cannot be captured);
 * nothing runs during the capture.  All pointers are device memory owned by
 * the caller and must outlive the graph; the graph is destroyed with
 * smcx_graph_destroy.  Errors: SMCX_E_INVALID_ARG, SMCX_E_NOT_READY before
 * smcx_set_epi, SMCX_E_HIP (capture failed).
 */
int smcx_ladder_capture(smcx_lattice *h, int32_t n_sweeps, uint64_t seed, const double *beta_dev,
                        uint32_t *sweep_counter_dev, int64_t *stats_dev, smcx_tie *ties_dev,
                        int32_t tie_cap, int32_t *tie_count_dev, void *stream, void **graph_out);

/*
 * Any sweep mode as a replayable graph.  Captures, on `stream`, the launches
 * of smcx_sweep(h, n_sweeps, seed, first, beta_dev, ...) in `mode`, where the
 * first sweep index is read from *sweep_counter_dev (device uint32) when the
 * graph runs and advanced by n_sweeps at its end, so every replay continues
 * the chain.  beta_dev: device double [n_sweeps][R], read at every replay.
 * The other arguments are as for smcx_sweep; *graph_out receives an
 * executable graph for smcx_graph_launch.  `stream` must be a created stream;
 * nothing runs during the capture; timing must be disabled.
 */
int smcx_sweep_capture(smcx_lattice *h, int32_t n_sweeps, uint64_t seed, const double *beta_dev,
                       uint32_t *sweep_counter_dev, int64_t *stats_dev, smcx_tie *ties_dev, int32_t tie_cap,
                       int32_t *tie_count_dev, int32_t mode, void *stream, void **graph_out);

int smcx_graph_launch(void *graph, void *stream);

int smcx_graph_destroy(void *graph);

/* Kernel timing for measurement: while enabled, every mini-step and
 * persistent sweep launch is bracketed with HIP events on its stream.
 * smcx_timing_read synchronises, returns the summed kernel time (ms) and the
 * number of timed launches since the last read, and resets both. */
int smcx_timing_enable(smcx_lattice *h, int32_t enable);
int smcx_timing_read(smcx_lattice *h, double *ms_out, int64_t *launches_out);

#ifdef __cplusplus
}
#endif

#endif /* SMCX_H */
