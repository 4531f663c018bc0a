// Device-visible data layouts shared by the host runtime and the kernels.
#pragma once
#include <stdint.h>

namespace sage {

constexpr uint32_t kBlock = 65536;      // bytes per read-only block
constexpr uint32_t kBlockShift = 16;

// FP64K-v1 key constants: low 32 bits of the first four splitmix64 outputs
// from state 0 (lowest bit set) and the fifth output (lowest bit set).
constexpr uint32_t kFpK0 = 0x7b1dcdafu;
constexpr uint32_t kFpK1 = 0xa1b965f5u;
constexpr uint32_t kFpK2 = 0x8009454fu;
constexpr uint32_t kFpK3 = 0x724c81edu;
constexpr uint64_t kFpK4 = 0x1b39896a51a8749bull;

// One block operation (same layout as sage_blk_op).
struct BlkOp {
  uint64_t src;
  uint64_t dst;
  uint32_t len;
  uint32_t op;  // 0 copy, 1 verify
};

// ---------------------------------------------------------------- MLP groups
// A grouped launch covers several functions of one MLP shape.  Group g owns
// rows [row0, row0 + m) of the launch's row space and the weight block table
// `wtab` (device address of each 64 KiB block of the function's blob).
struct GemmGroup {
  uint64_t wtab;        // const uint64_t* : block -> device address
  uint32_t m;           // rows
  uint32_t row0;        // first row in the launch's row space
  uint32_t tile_start;  // first tile of this group (prefix sum)
  uint32_t pad;
};

struct GemmHdr {
  uint32_t n_groups;
  uint32_t total_tiles;
  uint32_t total_rows;
  uint32_t pad;
};

// Per-layer arguments, passed by value.  A row r of the launch lives at
// a_tab ? a_tab[r] : a_base + r * K * elem (same for C with N).
struct LayerArgs {
  const uint64_t* a_tab;
  const uint8_t* a_base;
  const uint64_t* c_tab;
  uint8_t* c_base;
  uint64_t w_off;       // byte offset of this layer inside the blob
  uint32_t N, K;
  uint32_t flags;       // kRelu | kOutF32
  uint32_t pad;
};
constexpr uint32_t kRelu = 1u;
constexpr uint32_t kOutF32 = 2u;

// ---------------------------------------------------------------- stencil
struct StencilArgs {
  const uint64_t* ctab;   // coefficient blocks, or null: every cell uses `coef`
  const uint64_t* src;    // per field: device address of the sweep's input
  const uint64_t* dst;    // per field: device address of the sweep's output
  uint32_t nx, ny, nz;
  uint32_t n_fields;
  uint32_t tiles_x, tiles_y, tiles_z;  // spatial tiles per axis
  uint32_t spatial_tiles;              // tiles_x * tiles_y * tiles_z
  float coef;
};

// stencil7_sweep2 tile: cells along x, rows along y, planes along z marched
constexpr int kStencil2TX = 256, kStencil2TY = 16, kStencil2TZ = 64;

}  // namespace sage
