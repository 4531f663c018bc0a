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

// ---------------------------------------------------------------------------
// Two Jacobi sweeps per pass (temporal blocking): u0 is read and u2 written
// once for two sweeps; the intermediate u1 never leaves the workgroup.
//
// Output tile: 256 x-cells (x0 .. x0 + 255, lane l of a wave owns 4 of them,
// as in stencil7_sweep2) by kFusedRows y-rows (yo .. yo + 13) by kS2TZ
// planes.  The 16 waves hold rows yo - 1 + w (w = 0 .. 15): sweep 1 computes
// u1 on all 16 rows and on the two cells just outside the x range (lane 0
// of a wave: x0 - 1, lane 63: x0 + 256, one scalar each), sweep 2 computes u2
// on rows w = 1 .. 14 from those u1 values.  Tiles overlap by one row on
// each side in y (tiles step by 14 rows), and by one u1 cell on each side
// in x (computed twice, by both neighbours).
//
// The z march lags sweep 2 one plane behind sweep 1: iteration p computes
// u1 at plane p and u2 at plane p - 1.  Per plane one barrier: before it
// each wave publishes its u0 row of plane p (with the cells x0 - 1 and
// x0 + 256) in an LDS buffer; after it, sweep 1 reads the y neighbours of
// plane p and sweep 2 reads the u1 rows of plane p - 1 that every wave
// published after the previous barrier.  Both LDS buffers alternate by
// plane parity, so a buffer is rewritten only after a barrier that follows
// the last read of it.
//
// Each cell's arithmetic is the one of stencil7_sweep2 (the same operand
// order), so a pass equals two single sweeps bit for bit.  Cells on the
// grid boundary keep their value in both sweeps.
constexpr int kFusedRows = kS2Y - 2;  // output rows per tile
constexpr int kRowPad = 4;            // LDS row: [pad | x0 - 1 | 256 cells | x0 + 256 | pad]
constexpr int kRowLen = kS2X + 2 * kRowPad;

__device__ __forceinline__ float relax1(float centre, float xm, float xp, float ym, float yp, float zm, float zp,
                                        float c) {
  float sum = xm + xp;
  sum += ym;
  sum += yp;
  sum += zm;
  sum += zp;
  return centre + c * (sum * (1.0f / 6.0f) - centre);
}

extern "C" __global__ __launch_bounds__(1024) void stencil7_fused2(StencilArgs sa) {
  __shared__ __attribute__((aligned(16))) float r0[2][kS2Y + 2][kRowLen];  // u0 rows yo - 2 .. yo + 15
  __shared__ __attribute__((aligned(16))) float r1[2][kS2Y][kS2X];          // u1 rows yo - 1 .. yo + 14
  const uint32_t id = blockIdx.x;
  const uint32_t xcd = id & 7, q = id >> 3;
  const uint32_t f = q % sa.n_fields;
  const uint32_t s = (q / sa.n_fields) * 8 + xcd;
  if (s >= sa.spatial_tiles) return;  // whole workgroup
  const uint32_t tx = s % sa.tiles_x;
  const uint32_t ty = (s / sa.tiles_x) % sa.tiles_y;
  const uint32_t tz = s / (sa.tiles_x * sa.tiles_y);
  const int nx = (int)sa.nx, ny = (int)sa.ny, nz = (int)sa.nz;
  const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
  const int x0 = (int)tx * kS2X, x = x0 + 4 * lane;
  const int yo = (int)ty * kFusedRows, y = yo - 1 + w;
  const int z0 = (int)tz * kS2TZ, z1 = z0 + kS2TZ < nz ? z0 + kS2TZ : nz;
  const bool row_ok = y >= 0 && y < ny;
  const bool act = row_ok && x < nx;                        // this lane holds cells of a real row
  const bool out_row = w >= 1 && w <= kFusedRows && row_ok;  // sweep 2 writes this row
  const float* __restrict__ src = reinterpret_cast<const float*>(sa.src[f]);
  float* __restrict__ dst = reinterpret_cast<float*>(sa.dst[f]);
  const int64_t plane = (int64_t)nx * ny;
  const int64_t rowoff = (int64_t)y * nx + x;
  const f32x4 zero = f32x4{0.f, 0.f, 0.f, 0.f};
  // the u1 cells just outside the x range: lane 0 owns x0 - 1, lane 63 x0 + 256
  const bool ex_l = lane == 0 && row_ok && x0 > 0;
  const bool ex_r = lane == 63 && row_ok && x0 + kS2X < nx;
  const int ex_x = lane == 0 ? x0 - 1 : x0 + kS2X;
  const bool ex = ex_l || ex_r;
  const int64_t exoff = (int64_t)y * nx + ex_x;
  // halo rows of u0 outside the 16 held rows: wave 0 loads yo - 2, wave 15 yo + 15
  const int hy = w == 0 ? yo - 2 : yo + kFusedRows + 1;
  const bool halo = (w == 0 || w == kS2Y - 1) && hy >= 0 && hy < ny;
  const int hidx = w == 0 ? 0 : kS2Y + 1;
  const int64_t hoff = (int64_t)hy * nx + x, hexoff = (int64_t)hy * nx + ex_x;
  const bool hx = halo && x < nx, hex = halo && ((lane == 0 && x0 > 0) || (lane == 63 && x0 + kS2X < nx));

  const int ps = z0 > 0 ? z0 - 1 : 0;  // first u1 plane
  const int pe = z1;                   // last iteration (u1 only while p < nz)
  // u0 history of this lane's cells (planes p - 1, p, p + 1) and of its extra cell
  f32x4 um = (act && ps > 0) ? ld4(src + (int64_t)(ps - 1) * plane + rowoff) : zero;
  f32x4 uc = act ? ld4(src + (int64_t)ps * plane + rowoff) : zero;
  f32x4 up = (act && ps + 1 < nz) ? ld4(src + (int64_t)(ps + 1) * plane + rowoff) : zero;
  float em = (ex && ps > 0) ? ld1(src + (int64_t)(ps - 1) * plane + exoff) : 0.f;
  float ec = ex ? ld1(src + (int64_t)ps * plane + exoff) : 0.f;
  float ep = (ex && ps + 1 < nz) ? ld1(src + (int64_t)(ps + 1) * plane + exoff) : 0.f;
  // u1 history (planes p - 2, p - 1) of this lane's cells and of its extra cell, c of plane p - 1
  f32x4 v1m = zero, v1c = zero, cprev = zero;
  float e1c = 0.f;
  // Everything plane p needs besides the u0 history is loaded one iteration
  // ahead (the iteration is then bound by the barrier and the arithmetic,
  // not by the latency of these loads): the halo row and its outer cell,
  // the extra cell's outer x neighbour and the coefficients of plane p.
  // A coefficient's block-table entry for plane p + 1 is read with them,
  // its value one iteration later.
  const bool exo_ok = ex && (lane == 0 || ex_x + 1 < nx);
  const int64_t exo_off = exoff + (lane == 0 ? -1 : 1);  // u0 at x0 - 2 (lane 0) or x0 + 257 (lane 63)
  auto ctab_at = [&](int z, int xx) -> const uint8_t* {
    const uint64_t coff = ((uint64_t)z * ny + y) * nx * 4 + (uint64_t)xx * 4;
    return reinterpret_cast<const uint8_t*>(sa.ctab[coff >> kBlockShift]) + (coff & (kBlock - 1));
  };
  const bool cgrid = sa.ctab != nullptr;
  const f32x4 ccon = f32x4{sa.coef, sa.coef, sa.coef, sa.coef};
  f32x4 hnow = (hx && ps < nz) ? ld4(src + (int64_t)ps * plane + hoff) : zero;
  float henow = (hex && ps < nz) ? ld1(src + (int64_t)ps * plane + hexoff) : 0.f;
  float exonow = (exo_ok && ps < nz) ? ld1(src + (int64_t)ps * plane + exo_off) : 0.f;
  f32x4 cnow4 = (act && cgrid && ps < nz) ? *reinterpret_cast<const f32x4*>(ctab_at(ps, x)) : ccon;
  float cnow1 = (ex && cgrid && ps < nz) ? *reinterpret_cast<const float*>(ctab_at(ps, ex_x)) : sa.coef;
  const uint8_t* cp4 = (act && cgrid && ps + 1 < nz) ? ctab_at(ps + 1, x) : nullptr;    // plane p + 1
  const uint8_t* cp1 = (ex && cgrid && ps + 1 < nz) ? ctab_at(ps + 1, ex_x) : nullptr;
  uint32_t b = (uint32_t)ps & 1u;
  for (int p = ps; p <= pe; p++, b ^= 1u) {
    const bool have = p < nz;  // plane p exists: sweep 1 runs
    const int64_t pz = (int64_t)p * plane;
    const bool next = p + 1 < nz && p + 1 <= pe;  // plane p + 1 is visited
    // prefetch u0 of plane p + 2 (used two iterations from here)
    const f32x4 un = (act && p + 2 < nz && p + 1 <= pe) ? ld4(src + pz + 2 * plane + rowoff) : zero;
    const float en = (ex && p + 2 < nz && p + 1 <= pe) ? ld1(src + pz + 2 * plane + exoff) : 0.f;
    // prefetch what plane p + 1 needs
    const f32x4 hnext = (hx && next) ? ld4(src + pz + plane + hoff) : zero;
    const float henext = (hex && next) ? ld1(src + pz + plane + hexoff) : 0.f;
    const float exonext = (exo_ok && next) ? ld1(src + pz + plane + exo_off) : 0.f;
    const f32x4 cnext4 = cp4 && next ? *reinterpret_cast<const f32x4*>(cp4) : ccon;
    const float cnext1 = cp1 && next ? *reinterpret_cast<const float*>(cp1) : sa.coef;
    const uint8_t* cpn4 = (act && cgrid && p + 2 < nz && p + 1 <= pe) ? ctab_at(p + 2, x) : nullptr;
    const uint8_t* cpn1 = (ex && cgrid && p + 2 < nz && p + 1 <= pe) ? ctab_at(p + 2, ex_x) : nullptr;
    const float exo = exonow;
    // publish u0 rows of plane p (own cells + the cells just outside x)
    if (have) {
      *reinterpret_cast<f32x4*>(&r0[b][w + 1][kRowPad + 4 * lane]) = uc;
      if (ex) r0[b][w + 1][lane == 0 ? kRowPad - 1 : kRowPad + kS2X] = ec;
      if (hx) *reinterpret_cast<f32x4*>(&r0[b][hidx][kRowPad + 4 * lane]) = hnow;
      if (hex) r0[b][hidx][lane == 0 ? kRowPad - 1 : kRowPad + kS2X] = henow;
    }
    __syncthreads();
    // ---- sweep 1: u1 at plane p (shuffles by every lane of the wave)
    float left = __shfl_up(uc.w, 1, 64);
    float right = __shfl_down(uc.x, 1, 64);
    f32x4 v1 = uc;
    float e1 = ec;
    f32x4 cnow = zero;
    if (have && act) {
      const bool z_edge = p == 0 || p == nz - 1;
      if (!z_edge && y != 0 && y != ny - 1) {
        const f32x4 ym = *reinterpret_cast<const f32x4*>(&r0[b][w][kRowPad + 4 * lane]);
        const f32x4 yp = *reinterpret_cast<const f32x4*>(&r0[b][w + 2][kRowPad + 4 * lane]);
        if (lane == 0) left = r0[b][w + 1][kRowPad - 1];
        if (lane == 63) right = x + 4 < nx ? r0[b][w + 1][kRowPad + kS2X] : 0.f;
        cnow = cnow4;
        const float nb[4][2] = {{left, uc.y}, {uc.x, uc.z}, {uc.y, uc.w}, {uc.z, right}};
#pragma unroll
        for (int e = 0; e < 4; e++) {
          const int xe = x + e;
          if (xe == 0 || xe == nx - 1) continue;
          v1[e] = relax1(uc[e], nb[e][0], nb[e][1], ym[e], yp[e], um[e], up[e], cnow[e]);
        }
      }
    }
    if (have && ex) {
      const bool edge = p == 0 || p == nz - 1 || y == 0 || y == ny - 1 || ex_x == 0 || ex_x == nx - 1;
      if (!edge) {
        const int col = lane == 0 ? kRowPad - 1 : kRowPad + kS2X;
        const float inner = lane == 0 ? uc.x : uc.w;  // the own cell next to it
        const float xm = lane == 0 ? exo : inner, xp = lane == 0 ? inner : exo;
        e1 = relax1(ec, xm, xp, r0[b][w][col], r0[b][w + 2][col], em, ep, cnow1);
      }
    }
    // ---- sweep 2: u2 at plane p - 1 from u1 of planes p - 2, p - 1, p
    const int qz = p - 1;
    float left2 = __shfl_up(v1c.w, 1, 64);
    float right2 = __shfl_down(v1c.x, 1, 64);
    if (lane == 0) left2 = e1c;
    if (lane == 63) right2 = e1c;
    if (qz >= z0 && act && out_row) {
      f32x4 out = v1c;
      const bool z_edge = qz == 0 || qz == nz - 1;
      if (!z_edge && y != 0 && y != ny - 1) {
        const f32x4 ym = *reinterpret_cast<const f32x4*>(&r1[b ^ 1u][w - 1][4 * lane]);
        const f32x4 yp = *reinterpret_cast<const f32x4*>(&r1[b ^ 1u][w + 1][4 * lane]);
        const float nb[4][2] = {{left2, v1c.y}, {v1c.x, v1c.z}, {v1c.y, v1c.w}, {v1c.z, right2}};
        // u1 of plane p exists only while p < nz; at p == nz the plane p - 1 is a boundary plane
#pragma unroll
        for (int e = 0; e < 4; e++) {
          const int xe = x + e;
          if (xe == 0 || xe == nx - 1) continue;
          out[e] = relax1(v1c[e], nb[e][0], nb[e][1], ym[e], yp[e], v1m[e], v1[e], cprev[e]);
        }
      }
      st4(dst + (int64_t)qz * plane + rowoff, out);
    }
    // publish u1 rows of plane p for the next iteration's sweep 2
    if (have && act) *reinterpret_cast<f32x4*>(&r1[b][w][4 * lane]) = v1;
    v1m = v1c;
    v1c = v1;
    e1c = e1;
    cprev = cnow;
    um = uc;
    uc = up;
    up = un;
    em = ec;
    ec = ep;
    ep = en;
    hnow = hnext;
    henow = henext;
    exonow = exonext;
    cnow4 = cnext4;
    cnow1 = cnext1;
    cp4 = cpn4;
    cp1 = cpn1;
  }
}
