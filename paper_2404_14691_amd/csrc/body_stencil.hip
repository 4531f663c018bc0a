// Function body of the stencil kind, built as its own code object
// (sage_stencil.hsaco).
//
//   stencil7_sweep: one Jacobi sweep for every field of a launch,
//       u'_p = u_p + c_p * ((sum of 6 face neighbours) / 6 - u_p) inside,
//       u'_p = u_p on the boundary,
//   with the read-only coefficient grid c reached through its 64 KiB block
//   table (nx * 4 divides 65536, so an x-row of c never crosses a block).
//
// A workgroup is 64 x-cells by 4 y-rows and marches kStencilTZ planes along
// z, carrying the z-1 / z / z+1 values in registers; x and y neighbours come
// from the caches.  Fields sharing c are interleaved so that the workgroups
// of one spatial tile run on one XCD (ids are dealt to the 8 XCDs round
// robin), where c is read from HBM once and reused from that XCD's L2.
#include <hip/hip_runtime.h>

#include "layout.h"

using namespace sage;

extern "C" __global__ __launch_bounds__(256) void stencil7_sweep(StencilArgs sa) {
  const uint32_t id = blockIdx.x;
  const uint32_t xcd = id & 7, q = id >> 3;
  const uint32_t f = q % sa.n_fields;
  const uint32_t s = (q / sa.n_fields) * 8 + xcd;
  if (s >= sa.spatial_tiles) return;
  const uint32_t tx = s % sa.tiles_x;
  const uint32_t ty = (s / sa.tiles_x) % sa.tiles_y;
  const uint32_t tz = s / (sa.tiles_x * sa.tiles_y);
  const uint32_t nx = sa.nx, ny = sa.ny, nz = sa.nz;
  const uint32_t x = tx * kStencilTX + (threadIdx.x & 63);
  const uint32_t y = ty * kStencilTY + (threadIdx.x >> 6);
  if (x >= nx || y >= ny) return;
  const uint32_t z0 = tz * kStencilTZ;
  const uint32_t z1 = z0 + kStencilTZ < nz ? z0 + kStencilTZ : nz;

  const float* __restrict__ src = reinterpret_cast<const float*>(sa.src[f]);
  float* __restrict__ dst = reinterpret_cast<float*>(sa.dst[f]);
  const uint64_t plane = (uint64_t)nx * ny;
  uint64_t idx = (uint64_t)z0 * plane + (uint64_t)y * nx + x;
  const bool xy_edge = x == 0 || x == nx - 1 || y == 0 || y == ny - 1;

  float u_m = z0 > 0 ? src[idx - plane] : 0.f;
  float u_c = src[idx];
  for (uint32_t z = z0; z < z1; z++, idx += plane) {
    const float u_p = z + 1 < nz ? src[idx + plane] : 0.f;
    float out = u_c;
    if (!xy_edge && z != 0 && z != nz - 1) {
      float sum = src[idx - 1] + src[idx + 1];
      sum += src[idx - nx];
      sum += src[idx + nx];
      sum += u_m;
      sum += u_p;
      const uint64_t off = ((uint64_t)z * ny + y) * nx * 4;
      const float* crow = reinterpret_cast<const float*>(sa.ctab[off >> kBlockShift] + (off & (kBlock - 1)));
      const float c = crow[x];
      out = u_c + c * (sum * (1.0f / 6.0f) - u_c);
    }
    dst[idx] = out;
    u_m = u_c;
    u_c = u_p;
  }
}
