// Device tables of the matching kernels (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/ds3.h"

namespace ds3 {

struct MatchConst {
  int max_iters;
  float lambda0, lambda_min, step_tol, ang_tol, range_tol;
  int radius;
  double q_min;
};

// One decoded direction: queries (another view's points in the reference camera) against a reference.
struct MatchDir {
  int64_t ref_off;  // pixel offset of the reference in the ray-image buffer
  int64_t qry_off;  // pixel offset of the queries in their arena
  int64_t out_off;  // offset of the per-query idx in the temporary idx buffer
  int32_t Hr, Wr, Hq, Wq;
};

// One side of the mutual check: pixels of `self`, forward matches into `other` and back.
struct MutualDir {
  int64_t fwd_off, bwd_off;  // offsets in the temporary idx buffer (self->other, other->self)
  int64_t out_off;           // offset of the final idx / valid outputs (write_out only)
  const float* conf_self;    // confidences of self (pixel 0), written by the ray-image pass
  const float* conf_other;   // confidences of other (pixel 0)
  int32_t H_self, W_self, H_other, W_other;
  int32_t count_slot;        // nu counter index
  int32_t write_out;         // 1 for the j side of an edge
  int64_t part_off;          // first per-tile count of this side in the count partials
};

// Blocks are dealt to 8 bins (block b -> bin b mod 8, which the dispatcher places on XCD b mod 8);
// entries of bin x are [bin_start[x], bin_start[x+1]) with within-bin tile prefixes (one kMatchTile^2
// tile of query pixels per block for the matching, kMutualPx pixels for the mutual check).
struct ItemMap {
  const int32_t* bin_start;  // 9
  const int32_t* prefix;     // per entry: first tile of the entry within its bin
  const int32_t* bin_tiles;  // 8
};

int launch_raymap(const void* arena, int64_t n, ds3_dtype dt, float4* rays, float* conf, hipStream_t s);
int launch_match_one(const float4* rays, int H, int W, const void* qry, int Hq, int Wq, ds3_dtype dt,
                     const MatchConst& P, int32_t* idx_out, float* p_out, int32_t* it_out, hipStream_t s);
// LM step counting of the batched launch: per-block sums spread over kStepStripes counters, 128 B apart.
constexpr int kStepStripes = 256;
constexpr int kStripeStride = 32;
// step_stripes may be NULL (no counting); it must start at zero.
// Query tiles of the batched matching: kMatchTile x kMatchTile pixels, one block of 256 threads each.
constexpr int kMatchTile = 16;
inline int32_t match_tiles(int H, int W) {
  return int32_t(((H + kMatchTile - 1) / kMatchTile) * ((W + kMatchTile - 1) / kMatchTile));
}
int launch_match_batched(const float4* rays, const void* cross, ds3_dtype dt, const MatchDir* dirs,
                         ItemMap map, int grid, const MatchConst& P, int32_t* idx_tmp,
                         unsigned* step_stripes, hipStream_t s);
int launch_sum_stripes(const unsigned* step_stripes, unsigned long long* out, hipStream_t s);
int launch_mutual(const MutualDir* md, ItemMap map, int grid, ds3_dtype dt, const MatchConst& P,
                  const int32_t* idx_tmp, int32_t* idx_final, uint8_t* valid, unsigned* part,
                  hipStream_t s);
// Pixels per block of the mutual check (four per thread).
constexpr int kMutualPx = 1024;

// counts[slot] = sum of the per-tile partials [side[2 slot], side[2 slot] + side[2 slot + 1]), fixed order.
int launch_side_counts(const unsigned* part, const int64_t* side, int n_slots, unsigned* counts, hipStream_t s);
int launch_nu_finalize(const unsigned* counts, const int64_t* npx, int n_edges, double nu_min, float* nu,
                       int32_t* admit, hipStream_t s);

}  // namespace ds3
