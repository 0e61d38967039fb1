// Host-side launchers of the libsmcx kernels (defined in smcx_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "smcx_internal.h"

namespace smcx {

const void* sweep_kernel(int lattice, int K, bool persistent, int preset, int nbuf);
const void* row_kernel(int lattice, int K, int S, int block, int preset);
hipError_t launch_sweep(const void* kernel, dim3 grid, int block, size_t lds, hipStream_t st, const SweepArgs& a);
hipError_t set_sweep_lds_limit(const void* kernel, size_t lds);
hipError_t sweep_occupancy(const void* kernel, int block, size_t lds, int* blocks_per_cu);
// Natural layout <-> padded copy of replica r, or of every replica in one
// launch when r < 0 (nrows: the largest replica's rows, nrep replicas).
hipError_t launch_pack(int lattice, int K, bool unpack, bool planar, uint8_t* occ, uint8_t* ws,
                       const RepDev* reps, int r, int64_t nrows, int nrep, hipStream_t st);
hipError_t launch_validate(const uint8_t* occ, int64_t n, int K, int32_t* bad, hipStream_t st);
hipError_t launch_fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t st);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st);
hipError_t launch_advance_counter(uint32_t* counter, uint32_t n, hipStream_t st);
hipError_t launch_pair_counts(int lattice, int K, int S, const uint8_t* occ, int64_t N, const int32_t* L,
                              int B, int64_t* counts, hipStream_t st);
hipError_t launch_energy(const int64_t* C, const double* V, int R, int SKK, double* E, hipStream_t st);
// Device address of the static workspace on the current device (looked up
// once per device with that device current).
hipError_t static_workspace(void** ptr);
hipError_t launch_energy_grad(const int64_t* C, const double* g, int B, int SKK, double* grad, hipStream_t st);
// Largest qSRO affected set a trial can have (entries of its LDS terms).
constexpr int kQsroMaxAff = 256;
// Largest reach (cells per axis) of the windowed qSRO trial: a box of
// (2 reach + 1)^3 cells around the active site's cell.
constexpr int kQsroMaxReach = 4;

// Arguments of one qSRO mini-step launch over one replica.
struct QsroArgs {
    uint8_t* occ;          // this replica's occupancy (natural layout)
    int L0, L1, L2, K, S, Z1, sumZ, naff_max;
    const int32_t* org;    // cell origins: x (ncx + 1), y (ncy + 1), z (ncz + 1)
    int ncx, ncy, ncz;
    int o0, o1, o2, b;     // the mini-step's offsets and basis site
    int reach;             // cells from the active site's cell to the farthest site a trial reads, per axis
    uint32_t sweep, replica;
    uint64_t seed;
    double beta;
    const int32_t* aff;    // [m][Z1][1 + naff_max]: count, then packed displacements
    const int32_t* nbr;    // [m][sumZ]: packed neighbour displacements, shells in order
    const double* V;       // [S][K][K]
    const double* W;       // [S][K]
    const int32_t* Z;      // [S]
    int64_t* slots;        // [gridDim][3]: each workgroup's attempted / accepted / near-tie counts
    smcx_tie* ties;
    int32_t tie_cap;
    int32_t* tie_count;
};

hipError_t launch_qsro_ministep(int lattice, const QsroArgs& A, int grid, hipStream_t st);
hipError_t launch_qsro_reduce(const int64_t* slots, int n, int64_t* stats, hipStream_t st);
// workgroups of a qSRO mini-step launch (each has a counter slot)
constexpr int kQsroGrid = 8192;
hipError_t launch_local_energy(int lattice, const uint8_t* occ, const int32_t* L, int K, int S, const double* V,
                               double* e, hipStream_t st);
hipError_t launch_clusters(int lattice, const double* e, const int32_t* L, double threshold, int32_t* label,
                           int32_t* size, int64_t* n_clusters, hipStream_t st);
hipError_t launch_heat_capacity(const double* E, const double* beta_steps, const RepDev* reps, int n_steps, int n_rec,
                                int R, double* cv, hipStream_t st);
hipError_t launch_exchange(const double* E, const double* beta_slot, int32_t* rep_at, int R, uint64_t seed,
                           uint32_t round, double* beta_rows, int n_rows, int64_t* xstats, smcx_tie* ties,
                           int32_t tie_cap, int32_t* tie_count, hipStream_t st);

}  // namespace smcx
