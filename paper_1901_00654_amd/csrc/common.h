// Shared definitions of the tsmg device kernels and their host launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tsmg {

constexpr int kMaxDim = 5;
constexpr int kDeg = 3;          // cubic B-splines
constexpr int kBlock = 256;      // threads per workgroup for every kernel
// Most sorted points one workgroup of the point pass takes, by dimension
// (bounded by the LDS that stages them).
constexpr int kMaxPointsPerBlock[kMaxDim + 1] = {0, 2048, 2048, 1024, 1024, 512};
// Tile side 2^kTileBits[d] cells per dimension in the point pass (levels with
// fewer cells use the whole grid as one tile).
constexpr int kTileBits[kMaxDim + 1] = {0, 6, 4, 2, 1, 1};

// What the point pass of the data term computes (Alg. 3/4/5):
enum DataMode : int {
  kApply = 0,   // out += Phi'(Phi c)           gather then scatter
  kRhs = 1,     // out += Phi' y                scatter of the responses
  kDiag = 2,    // out += sum_i v_i[k]^2        Alg. 5
};

// Per-launch description of one level of one problem for the point pass.
struct DataArgs {
  const void* tfrac;        // [d][n] T: position inside the finest knot cell, in [0,1]
  const uint32_t* cell;     // [n] finest-level cell, C order (N_G^(d-1-p) weights)
  const uint32_t* mkey;     // [n] finest-level cell, Morton order (the sort key)
  const double* y;          // [n] responses (kRhs only)
  const int32_t* off;       // [N_G^d + 1] first sorted point of each finest Morton cell
  const void* c;            // [K_g] T, coefficient vector (kApply only)
  void* out;                // [K_g] T, accumulated atomically
  int64_t n;                // number of points
  int G;                    // finest level (N_G = 2^G)
  int g;                    // this level
  int tb;                   // tile side 2^tb level-g cells per dimension (tb <= g)
  int ppb;                  // points per workgroup (<= kMaxPointsPerBlock[d])
  // Optional work list of this level, built once at setup (null: each
  // workgroup takes ppb points and derives its tile segments and items from
  // mkey and off on the fly). With a work list a workgroup takes whole tile
  // segments - up to several chunks of at most ppb points each - staging the
  // coefficient patch and flushing the accumulator once per segment.
  const int32_t* wl_first;  // [workgroups + 1] first chunk of each workgroup
  const int4* wl_chunks;    // [chunks + 1] {first point, end point, first item,
                            //  tile | kChunkFirst | kChunkLast (of its segment)}
  const uint32_t* wl_items; // [items] cell in tile | first point - chunk start << 8 | count << 20
  int wl_groups;            // workgroups of the work list
  // Run-to-run reproducible form (needs the work list, every chunk of which
  // is a whole segment): the point pass stores each chunk's patch (FP64,
  // (2^tb + 3)^d entries) to det_part[chunk] and k_det_reduce adds, per
  // coefficient, the patches of the tiles covering it in a fixed order.
  int det;
  double* det_part;          // [chunks][patch]
  const int32_t* det_tile_first;   // [tiles + 1] first chunk of each tile (Morton order)
};
constexpr uint32_t kChunkFirst = 1u << 31;   // first chunk of a tile segment
constexpr uint32_t kChunkLast = 1u << 30;    // last chunk of a tile segment
constexpr uint32_t kChunkTile = kChunkLast - 1u;

// Points per item (a cell's run of points given to one lane group), by d.
constexpr int kItemQ[kMaxDim + 1] = {0, 16, 16, 8, 16, 32};

// Packing of one work-list item (a cell's run of at most Q points).
constexpr int kItemLoShift = 8;
constexpr int kItemCntShift = 20;

}  // namespace tsmg
