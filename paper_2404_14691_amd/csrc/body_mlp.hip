// Function bodies of the MLP kinds, built as a separate code object
// (sage_mlp.hsaco) that fn_register loads with hipModuleLoad while the
// function's weights are moving to the device.
//
//   ggemm_bf16_<BM>x<BN>: one layer of a grouped BF16 MLP,
//       C[r, n] = act(sum_k A[r, k] * W[n, k]) for every row r of every group,
//       A and W BF16, FP32 accumulation with v_mfma_f32_16x16x32_bf16.
//       Persistent: each workgroup walks tiles blockIdx.x, +gridDim.x, ...
//       over a tile list spanning all groups (ragged rows per group).
//       W rows are found through the function's 64 KiB block table.
//   mlp_f32_layer: the same layer in FP32 on the vector ALUs for small
//       batches (one wave per two output columns, fixed reduction order).
//
// Every tile shape walks K in the same order with the same MFMA, so an
// output element's bits do not depend on the tile shape, on its row
// position or on which other rows share the launch.
#include <hip/hip_runtime.h>

#include "layout.h"

using namespace sage;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const u32x4 g_u32x4;  // global (not flat) loads

namespace {

constexpr int BK = 64;             // K per LDS stage (two MFMA K-steps of 32)
constexpr int kRowBytes = BK * 2;  // 128 B of a row per stage = 8 chunks of 16 B

__device__ __forceinline__ uint32_t find_group(const GemmGroup* groups, uint32_t n, uint32_t tile) {
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (groups[mid].tile_start <= tile) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ const uint8_t* a_row(const LayerArgs& la, uint32_t r, uint32_t esize) {
  return la.a_tab ? reinterpret_cast<const uint8_t*>(la.a_tab[r]) : la.a_base + (uint64_t)r * la.K * esize;
}

__device__ __forceinline__ uint8_t* c_row(const LayerArgs& la, uint32_t r, uint32_t esize) {
  return la.c_tab ? reinterpret_cast<uint8_t*>(la.c_tab[r]) : la.c_base + (uint64_t)r * la.N * esize;
}

// LDS byte offset of 16-byte chunk `c` of row `r` in a [rows][BK] stage:
// chunks are XOR-swizzled by the row so that 8 lanes reading one chunk
// column of 8 consecutive rows hit 8 different bank groups.
__device__ __forceinline__ uint32_t swz(uint32_t r, uint32_t c) { return r * kRowBytes + ((c ^ (r & 7)) << 4); }

// Global -> registers: NL 16-byte chunks per thread for one K stage.
template <int NL, int NCH>
__device__ __forceinline__ void gload(u32x4 (&r)[NL], const uint8_t* const (&p)[NL], uint32_t kt, uint32_t t) {
#pragma unroll
  for (int i = 0; i < NL; i++)
    if (NCH % 256 == 0 || t + 256 * i < (uint32_t)NCH)
      r[i] = *(g_u32x4*)(uintptr_t)(p[i] + kt * kRowBytes);
}

// Registers -> one LDS stage (swizzled rows).
template <int NL, int NCH>
__device__ __forceinline__ void sstore(uint8_t* stage, const u32x4 (&r)[NL], uint32_t t, uint32_t chunk) {
#pragma unroll
  for (int i = 0; i < NL; i++)
    if (NCH % 256 == 0 || t + 256 * i < (uint32_t)NCH)
      *reinterpret_cast<u32x4*>(stage + swz((t >> 3) + 32 * i, chunk)) = r[i];
}

template <int BM, int BN, int WM, int WN>
__device__ __forceinline__ void ggemm_bf16(const GemmHdr* __restrict__ hdr, const GemmGroup* __restrict__ groups,
                                           const LayerArgs la, uint8_t* lds) {
  constexpr int NWN = BN / WN, NWM = BM / WM;
  static_assert(NWN * NWM == 4, "four waves per workgroup");
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int A_CH = BM * 8, B_CH = BN * 8;               // 16-B chunks per stage
  constexpr int A_LD = (A_CH + 255) / 256, B_LD = (B_CH + 255) / 256;
  constexpr uint32_t A_STAGE = BM * kRowBytes, B_STAGE = BN * kRowBytes;
  uint8_t* const As = lds;                 // [2][BM][BK]
  uint8_t* const Bs = lds + 2 * A_STAGE;   // [2][BN][BK]

  const uint32_t t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const uint32_t wm = wave / NWN, wn = wave % NWN;
  const uint32_t N = la.N, K = la.K;
  const uint32_t total = hdr->total_tiles, G = hdr->n_groups;
  const uint32_t ld_chunk = t & 7;
  const bool out_f32 = la.flags & kOutF32, relu = la.flags & kRelu;
  const uint32_t KT = K / BK;

  for (uint32_t tile = blockIdx.x; tile < total; tile += gridDim.x) {
    const GemmGroup gr = groups[find_group(groups, G, tile)];
    const uint32_t local = tile - gr.tile_start;
    const uint32_t m_tiles = (gr.m + BM - 1) / BM;
    const uint32_t m0 = (local % m_tiles) * BM, n0 = (local / m_tiles) * BN;
    const uint64_t* wtab = reinterpret_cast<const uint64_t*>(gr.wtab);

    const uint8_t* ap[A_LD];
    const uint8_t* bp[B_LD];
#pragma unroll
    for (int i = 0; i < A_LD; i++) {
      const uint32_t row = (t >> 3) + 32 * i;
      uint32_t r = m0 + (row < BM ? row : 0);
      r = r < gr.m ? r : gr.m - 1;  // ragged tail: reload a valid row, never stored
      ap[i] = a_row(la, gr.row0 + r, 2) + ld_chunk * 16;
    }
#pragma unroll
    for (int i = 0; i < B_LD; i++) {
      const uint32_t row = (t >> 3) + 32 * i;
      const uint64_t off = la.w_off + (uint64_t)(n0 + (row < BN ? row : 0)) * K * 2;
      bp[i] = reinterpret_cast<const uint8_t*>(wtab[off >> kBlockShift]) + (off & (kBlock - 1)) + ld_chunk * 16;
    }

    f32x4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; i++)
#pragma unroll
      for (int j = 0; j < FN; j++) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    u32x4 ra[A_LD], rb[B_LD];
    gload<A_LD, A_CH>(ra, ap, 0, t);
    gload<B_LD, B_CH>(rb, bp, 0, t);
    sstore<A_LD, A_CH>(As, ra, t, ld_chunk);
    sstore<B_LD, B_CH>(Bs, rb, t, ld_chunk);
    __syncthreads();
    for (uint32_t kt = 0; kt < KT; kt++) {
      const uint32_t cur = kt & 1;
      if (kt + 1 < KT) {
        gload<A_LD, A_CH>(ra, ap, kt + 1, t);
        gload<B_LD, B_CH>(rb, bp, kt + 1, t);
      }
#pragma unroll
      for (int ks = 0; ks < 2; ks++) {
        const uint32_t chunk = ks * 4 + (lane >> 4);
        bf16x8 af[FM], bfr[FN];
#pragma unroll
        for (int i = 0; i < FM; i++) {
          const uint32_t r = wm * WM + i * 16 + (lane & 15);
          af[i] = *reinterpret_cast<const bf16x8*>(As + cur * A_STAGE + swz(r, chunk));
        }
#pragma unroll
        for (int j = 0; j < FN; j++) {
          const uint32_t r = wn * WN + j * 16 + (lane & 15);
          bfr[j] = *reinterpret_cast<const bf16x8*>(Bs + cur * B_STAGE + swz(r, chunk));
        }
#pragma unroll
        for (int i = 0; i < FM; i++)
#pragma unroll
          for (int j = 0; j < FN; j++)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
      }
      if (kt + 1 < KT) {
        sstore<A_LD, A_CH>(As + (cur ^ 1) * A_STAGE, ra, t, ld_chunk);
        sstore<B_LD, B_CH>(Bs + (cur ^ 1) * B_STAGE, rb, t, ld_chunk);
      }
      __syncthreads();
    }

    // epilogue: lane holds column (lane & 15), rows 4*(lane >> 4) + 0..3 of each 16x16 fragment
#pragma unroll
    for (int i = 0; i < FM; i++) {
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const uint32_t r = m0 + wm * WM + i * 16 + 4 * (lane >> 4) + q;
        if (r < gr.m) {
          uint8_t* crow = c_row(la, gr.row0 + r, out_f32 ? 4 : 2);
#pragma unroll
          for (int j = 0; j < FN; j++) {
            const uint32_t col = n0 + wn * WN + j * 16 + (lane & 15);
            float v = acc[i][j][q];
            if (relu) v = v > 0.f ? v : 0.f;
            if (out_f32) reinterpret_cast<float*>(crow)[col] = v;
            else reinterpret_cast<__bf16*>(crow)[col] = (__bf16)v;
          }
        }
      }
    }
  }
}

}  // namespace

#define SAGE_GGEMM(BM, BN, WM, WN, OCC)                                                               \
  extern "C" __global__ __launch_bounds__(256, OCC) void ggemm_bf16_##BM##x##BN(                       \
      const GemmHdr* __restrict__ hdr, const GemmGroup* __restrict__ groups, LayerArgs la) {           \
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * (BM + BN) * kRowBytes];                    \
    ggemm_bf16<BM, BN, WM, WN>(hdr, groups, la, lds);                                                  \
  }

SAGE_GGEMM(16, 64, 16, 16, 2)
SAGE_GGEMM(32, 64, 16, 32, 2)
SAGE_GGEMM(32, 128, 32, 32, 2)
SAGE_GGEMM(64, 128, 32, 64, 2)
SAGE_GGEMM(128, 128, 64, 64, 2)
SAGE_GGEMM(256, 128, 128, 64, 1)
SAGE_GGEMM(128, 256, 64, 128, 1)

// ---------------------------------------------------------------- FP32 MLP
// Tiles: (group, block of 8 output columns); wave w of the workgroup owns
// columns 8*cb + 2w and 8*cb + 2w + 1 and walks the group's rows 8 at a
// time.  Lane l accumulates k = 4l + 256i (i = 0, 1, ...) with fmaf in order,
// then a fixed xor-butterfly sums the lanes.
extern "C" __global__ __launch_bounds__(256) void mlp_f32_layer(const GemmHdr* __restrict__ hdr,
                                                                const GemmGroup* __restrict__ groups,
                                                                LayerArgs la) {
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t K = la.K;
  const bool relu = la.flags & kRelu;
  for (uint32_t tile = blockIdx.x; tile < hdr->total_tiles; tile += gridDim.x) {
    const GemmGroup gr = groups[find_group(groups, hdr->n_groups, tile)];
    const uint32_t n = (tile - gr.tile_start) * 8 + wave * 2;
    const uint64_t* wtab = reinterpret_cast<const uint64_t*>(gr.wtab);
    const uint64_t off0 = la.w_off + (uint64_t)n * K * 4, off1 = off0 + (uint64_t)K * 4;
    const float* w0 = reinterpret_cast<const float*>(wtab[off0 >> kBlockShift] + (off0 & (kBlock - 1)));
    const float* w1 = reinterpret_cast<const float*>(wtab[off1 >> kBlockShift] + (off1 & (kBlock - 1)));
    for (uint32_t r0 = 0; r0 < gr.m; r0 += 8) {
      const uint32_t nr = gr.m - r0 < 8 ? gr.m - r0 : 8;
      const float* ar[8];
#pragma unroll
      for (int i = 0; i < 8; i++)
        ar[i] = reinterpret_cast<const float*>(a_row(la, gr.row0 + r0 + ((uint32_t)i < nr ? i : 0), 4));
      float acc0[8], acc1[8];
#pragma unroll
      for (int i = 0; i < 8; i++) acc0[i] = acc1[i] = 0.f;
      for (uint32_t k = lane * 4; k < K; k += 256) {
        const float4 wa = *reinterpret_cast<const float4*>(w0 + k);
        const float4 wb = *reinterpret_cast<const float4*>(w1 + k);
#pragma unroll
        for (int i = 0; i < 8; i++) {
          if ((uint32_t)i < nr) {
            const float4 a = *reinterpret_cast<const float4*>(ar[i] + k);
            acc0[i] = fmaf(a.x, wa.x, acc0[i]);
            acc0[i] = fmaf(a.y, wa.y, acc0[i]);
            acc0[i] = fmaf(a.z, wa.z, acc0[i]);
            acc0[i] = fmaf(a.w, wa.w, acc0[i]);
            acc1[i] = fmaf(a.x, wb.x, acc1[i]);
            acc1[i] = fmaf(a.y, wb.y, acc1[i]);
            acc1[i] = fmaf(a.z, wb.z, acc1[i]);
            acc1[i] = fmaf(a.w, wb.w, acc1[i]);
          }
        }
      }
#pragma unroll
      for (int i = 0; i < 8; i++) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          acc0[i] += __shfl_xor(acc0[i], o, 64);
          acc1[i] += __shfl_xor(acc1[i], o, 64);
        }
      }
      if (lane == 0) {
        for (uint32_t i = 0; i < nr; i++) {
          float* crow = reinterpret_cast<float*>(c_row(la, gr.row0 + r0 + i, 4));
          float v0 = acc0[i], v1 = acc1[i];
          if (relu) {
            v0 = v0 > 0.f ? v0 : 0.f;
            v1 = v1 > 0.f ? v1 : 0.f;
          }
          crow[n] = v0;
          crow[n + 1] = v1;
        }
      }
    }
  }
}
