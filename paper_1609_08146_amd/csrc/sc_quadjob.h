// sc_quadjob.h -- the work description shared by the quadrature kernel
// (sc_quad.hip) and the host code that builds it.  Not part of the public ABI.
#pragma once

#include <stdint.h>

namespace sc {

// One problem instance as seen by the quadrature kernel.  All pointers are
// device pointers.  Tiles of a job are numbered
//   local = (k * n_chunks + chunk) * obs_blocks + obs_block
// so that waves running side by side share (k, chunk) table data.
struct QuadJob {
    const void *tab;      // [n_k][n_tot][8] real (float or double); factored: [n_k][n_tot][4] real
    const void *pos;      // [n_tot][4] real; factored: [n_tot][8] real
    const void *obs;      // [n_obs_pad][4] real
    const void *hinv;     // [n_tot] 1 / (2|r_s|) real (general layout, series_delta)
    const void *beta;     // [n_tot] real (factored layout with the tied charge): rho_t = -i beta s / k
    const void *tabp;     // [n_k][n_tot][2] float (FP32 split form, tied charge): (|s|, arg(s) / 2 pi)
    const double *k;      // [n_k]
    void *partial;        // [n_chunks][n_k][n_obs_pad / 64][12][64] real
    int n_tot;            // surface + rim nodes
    int n_obs_pad;        // observation points, padded to the obs block
    int n_k;
    int chunk;            // nodes per split-K chunk
    int n_chunks;
    int obs_blocks;       // n_obs_pad / (64 * obs_per_lane)
    int factored;         // split form (FP32 or FP64) with the current factored as J~ = u s (u real, per node)
    int tied;             // factored, and the charge tied to the current: rho_t = -i beta s / k (beta real,
                          // per node); the B sums then carry 1/k, so the reduction drops its own 1/k
    int raw_phase;        // FP32 split form: |k delta| / 2 pi < 250 turns for every pair of the job
    int series_delta;     // split forms: |r'| <= 4e-4 |r_s| for every pair (delta and 1/|R| by series)
    int64_t tile0;        // first global tile of this job in the launch
    int64_t tile_offset;  // first job-local tile covered (a launch may cover a sub-range)
    int64_t n_tiles;      // tiles covered by this launch
};

enum QuadMode { MODE_FP64 = 0, MODE_SPLIT = 1, MODE_NAIVE = 2 };

// Work counters of one quadrature launch (one per XCD-sized segment of the tile list).
constexpr int QUAD_SEGMENTS = 8;

}  // namespace sc
