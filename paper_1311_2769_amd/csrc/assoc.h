// Hit association (assoc.hip), called from the C ABI in api.hip.
#pragma once

#include "hough_impl.h"

namespace hough {

// Bitmap dwords per (d0, phi0) row of the association's candidate bitmap.
int64_t assoc_row_words(int32_t n_kappa);

// Azimuth buckets of the hit order the association works in.
constexpr int kAssocBuckets = 1024;

// Hit association of one event: map is the context's [cells] int32 cell map,
// bits its [n_d0 * n_phi * assoc_row_words(n_kappa)] candidate bitmap,
// sorted room for n_hits hit records, hist kAssocBuckets int32, n_pairs an
// 8-byte counter; all are cleared or written here.  approx: the phi0 table
// holds the bin centres, so the bins may take the vote's approximate form
// with exact redos (when the grid has a near band).
hipError_t launch_associate(const GridArgs &g, const float *x, const float *y, int32_t n_hits, const Cand *cands,
                            const int32_t *n_found, int32_t cands_cap, int32_t min_votes, int32_t *map, uint32_t *bits,
                            float4 *sorted, int32_t *hist, int32_t *pairs, int64_t cap,
                            unsigned long long *n_pairs, bool approx, hipStream_t stream);

}  // namespace hough
