// Function body of the grid kinds, built as its own code object
// (sage_stencil.hsaco).
//
//   stencil7_sweep2: one Jacobi sweep for every field of a launch,
//       u'_p = u_p + c_p * ((sum of 6 face neighbours) / 6 - u_p) inside,
//       u'_p = u_p on the boundary,
//   with the read-only coefficient grid c reached through its 64 KiB block
//   table (nx * 4 divides 65536, so an x-row of c never crosses a block), or,
//   for the relaxation kind without read-only data, one constant c.
//
// Fields sharing c are interleaved so that the workgroups of one spatial
// tile run on one XCD (ids are dealt to the 8 XCDs round robin), where c is
// read from HBM once and reused from that XCD's L2.
#include <hip/hip_runtime.h>

#include "layout.h"

using namespace sage;

// 2.5D-blocked sweep.  A workgroup of 16 waves owns 256 x-cells by 16 y-rows
// and marches kStencil2TZ planes along z.  Lane l of wave w holds the four
// cells x0 + 4l .. x0 + 4l + 3 of row y0 + w (one 16-byte load):
//   x neighbours  - the adjacent lanes' registers (wave shuffles); the two
//                   cells just outside the wave's 256 come from memory;
//   y neighbours  - each wave publishes its plane-z row in LDS (double
//                   buffered, one barrier per plane); waves 0 and 15 also
//                   load the rows just outside the tile;
//   z neighbours  - registers (planes z - 1, z, z + 1, and z + 2 in flight).
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kS2X = kStencil2TX, kS2Y = kStencil2TY, kS2TZ = kStencil2TZ;

// Field data streams through once per sweep: nontemporal loads and stores
// keep it from evicting the shared coefficient grid, which the workgroups of
// all fields of a spatial tile read from the same XCD's L2.
__device__ __forceinline__ f32x4 ld4(const float* p) {
  return __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
}
__device__ __forceinline__ float ld1(const float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void st4(float* p, f32x4 v) { __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(p)); }

extern "C" __global__ __launch_bounds__(1024) void stencil7_sweep2(StencilArgs sa) {
  __shared__ __attribute__((aligned(16))) float rows[2][kS2Y + 2][kS2X];
  const uint32_t id = blockIdx.x;
  const uint32_t xcd = id & 7, q = id >> 3;
  const uint32_t f = q % sa.n_fields;
  const uint32_t s = (q / sa.n_fields) * 8 + xcd;
  if (s >= sa.spatial_tiles) return;  // whole workgroup: no barrier is left waiting
  const uint32_t tx = s % sa.tiles_x;
  const uint32_t ty = (s / sa.tiles_x) % sa.tiles_y;
  const uint32_t tz = s / (sa.tiles_x * sa.tiles_y);
  const uint32_t nx = sa.nx, ny = sa.ny, nz = sa.nz;
  const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t x0 = tx * kS2X, x = x0 + 4 * lane, y0 = ty * kS2Y, y = y0 + w;
  const uint32_t z0 = tz * kS2TZ, z1 = z0 + kS2TZ < nz ? z0 + kS2TZ : nz;
  const bool act = x < nx && y < ny;                 // this lane holds cells
  const float* __restrict__ src = reinterpret_cast<const float*>(sa.src[f]);
  float* __restrict__ dst = reinterpret_cast<float*>(sa.dst[f]);
  const uint64_t plane = (uint64_t)nx * ny;
  const uint64_t rowoff = (uint64_t)y * nx + x;
  const f32x4 zero = f32x4{0.f, 0.f, 0.f, 0.f};
  // halo cells outside this wave's x range, and halo rows outside the tile
  const bool need_xl = lane == 0 && act && x > 0;
  const bool need_xr = act && (x + 4 < nx) && (lane == 63 || x + 4 >= x0 + kS2X);
  const bool halo_lo = w == 0 && y0 > 0 && x < nx;
  const bool halo_hi = w == kS2Y - 1 && y0 + kS2Y < ny && x < nx;
  const uint64_t lo_off = ((uint64_t)(y0 - 1) * nx + x), hi_off = ((uint64_t)(y0 + kS2Y) * nx + x);

  f32x4 um = (act && z0 > 0) ? ld4(src + (uint64_t)(z0 - 1) * plane + rowoff) : zero;
  f32x4 uc = act ? ld4(src + (uint64_t)z0 * plane + rowoff) : zero;
  f32x4 up = (act && z0 + 1 < nz) ? ld4(src + (uint64_t)(z0 + 1) * plane + rowoff) : zero;
  uint32_t b = 0;
  for (uint32_t z = z0; z < z1; z++, b ^= 1) {
    const uint64_t pz = (uint64_t)z * plane;
    // plane z + 2 is loaded now and used two iterations from here
    const f32x4 un = (act && z + 2 < nz && z + 1 < z1) ? ld4(src + pz + 2 * plane + rowoff) : zero;
    const float xl = need_xl ? ld1(src + pz + rowoff - 1) : 0.f;
    const float xr = need_xr ? ld1(src + pz + rowoff + 4) : 0.f;
    const bool z_edge = z == 0 || z == nz - 1;
    *reinterpret_cast<f32x4*>(&rows[b][w + 1][4 * lane]) = uc;
    if (halo_lo) *reinterpret_cast<f32x4*>(&rows[b][0][4 * lane]) = ld4(src + pz + lo_off);
    if (halo_hi) *reinterpret_cast<f32x4*>(&rows[b][kS2Y + 1][4 * lane]) = ld4(src + pz + hi_off);
    __syncthreads();
    const f32x4 ym = *reinterpret_cast<const f32x4*>(&rows[b][w][4 * lane]);
    const f32x4 yp = *reinterpret_cast<const f32x4*>(&rows[b][w + 2][4 * lane]);
    float left = __shfl_up(uc.w, 1, 64);
    float right = __shfl_down(uc.x, 1, 64);
    if (lane == 0) left = xl;
    if (need_xr && lane == 63) right = xr;
    if (act) {
      f32x4 out = uc;
      if (!z_edge && y != 0 && y != ny - 1) {
        const uint64_t coff = ((uint64_t)z * ny + y) * nx * 4 + (uint64_t)x * 4;  // byte offset of c(x, y, z)
        const f32x4 c = sa.ctab ? *reinterpret_cast<const f32x4*>(sa.ctab[coff >> kBlockShift] + (coff & (kBlock - 1)))
                                : f32x4{sa.coef, sa.coef, sa.coef, sa.coef};
        const float nb[4][2] = {{left, uc.y}, {uc.x, uc.z}, {uc.y, uc.w}, {uc.z, right}};
#pragma unroll
        for (int e = 0; e < 4; e++) {
          const uint32_t xe = x + e;
          if (xe == 0 || xe == nx - 1) continue;
          float sum = nb[e][0] + nb[e][1];
          sum += ym[e];
          sum += yp[e];
          sum += um[e];
          sum += up[e];
          out[e] = uc[e] + c[e] * (sum * (1.0f / 6.0f) - uc[e]);
        }
      }
      st4(dst + pz + rowoff, out);
    }
    um = uc;
    uc = up;
    up = un;
  }
}
