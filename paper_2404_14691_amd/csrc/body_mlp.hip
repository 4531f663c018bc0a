// Function bodies of the MLP kinds, built as a separate code object
// (sage_mlp.hsaco) that fn_register loads with hipModuleLoad while the
// function's weights are moving to the device.
//
// One layer of a grouped BF16 MLP,
//     C[r, n] = act(sum_k A[r, k] * W[n, k]) for every row r of every group,
// A and W BF16, FP32 accumulation with v_mfma_f32_16x16x32_bf16, is one
// persistent kernel over a tile list that spans all groups (ragged rows per
// group); W rows are found through the function's 64 KiB block table.
// Tile-shape families (the launch planner picks among them):
//   ggemm_bf16_<BM>x<BN>   register-staged double-buffered LDS tiles;
//   ggemm2_bf16_<BM>x<BN>  the same, 8 waves, XCD-aware tile ranges;
//   ggemm3*_bf16_<BM>x<BN> direct-to-LDS loads into a ring of K slices,
//                          thin tiles for a few rows;
//   ggemm6*_bf16_<BM>x<BN> 8-wave ping-pong over the same ring, the main
//                          shape of large grouped launches.
// mlp_f32_layer is the same layer in FP32 on the vector ALUs for small
// batches (K split over a workgroup's waves, fixed reduction order).
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

template <int CTRL>
__device__ __forceinline__ float quad_swap(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), CTRL, 0xF, 0xF, false));
}

// Epilogue of every shape.  Lane l holds column l & 15 and rows
// 4 (l >> 4) + 0..3 of each 16 x 16 fragment; after relu, two DPP swaps
// (lanes l ^ 1, then l ^ 2) transpose each lane quad's 4 x 4 block, so that
// a lane holds 4 consecutive columns of one row and stores them at once
// (8 B of BF16 or 16 B of FP32): a quarter of the store instructions of
// one value per lane.  Values and rounding are unchanged.  Every lane of
// the wave runs the swaps; only the stores are bounded by the group's rows.
template <int FM, int FN>
__device__ __forceinline__ void store_tile(const f32x4 (&acc)[FM][FN], const LayerArgs& la, const GemmGroup& gr,
                                           uint32_t row_base, uint32_t col_base, bool relu, bool out_f32,
                                           uint32_t lane) {
  typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
  const bool b = lane & 1, hb = (lane >> 1) & 1;
  const uint32_t rq = row_base + 4 * (lane >> 4) + (lane & 3);  // this lane's row in each 16-row fragment
  const uint32_t cq = col_base + 4 * ((lane & 15) >> 2);        // its first column in each 16-column fragment
#pragma unroll
  for (int i = 0; i < FM; i++) {
    const uint32_t r = rq + i * 16;
    uint8_t* crow = r < gr.m ? c_row(la, gr.row0 + r, out_f32 ? 4 : 2) : nullptr;
#pragma unroll
    for (int j = 0; j < FN; j++) {
      f32x4 v = acc[i][j];
      if (relu) {
#pragma unroll
        for (int q = 0; q < 4; q++) v[q] = v[q] > 0.f ? v[q] : 0.f;
      }
      // quad lane c holds rows 0..3 of column c; after the swaps lane c holds row c, columns 0..3
      const float r0 = quad_swap<0xB1>(b ? v[0] : v[1]), r2 = quad_swap<0xB1>(b ? v[2] : v[3]);  // quad_perm [1,0,3,2]
      const float own0 = b ? v[1] : v[0], own2 = b ? v[3] : v[2];
      const float w00 = b ? r0 : own0, w01 = b ? own0 : r0, w10 = b ? r2 : own2, w11 = b ? own2 : r2;
      const float u0 = quad_swap<0x4E>(hb ? w00 : w10), u1 = quad_swap<0x4E>(hb ? w01 : w11);     // quad_perm [2,3,0,1]
      const float k0 = hb ? w10 : w00, k1 = hb ? w11 : w01;
      const float c0 = hb ? u0 : k0, c1 = hb ? u1 : k1, c2 = hb ? k0 : u0, c3 = hb ? k1 : u1;
      if (crow) {
        const uint32_t col = cq + j * 16;
        if (out_f32) *reinterpret_cast<f32x4*>(reinterpret_cast<float*>(crow) + col) = f32x4{c0, c1, c2, c3};
        else *reinterpret_cast<bf16x4*>(reinterpret_cast<__bf16*>(crow) + col) = bf16x4{(__bf16)c0, (__bf16)c1, (__bf16)c2, (__bf16)c3};
      }
    }
  }
}

// LDS byte offset of 16-byte chunk `c` of row `r` in a [rows][BK] stage:
// chunks are XOR-swizzled by the row so that 8 lanes reading one chunk
// column of 8 consecutive rows hit 8 different bank groups.
__device__ __forceinline__ uint32_t swz(uint32_t r, uint32_t c) { return r * kRowBytes + ((c ^ (r & 7)) << 4); }

// Global -> registers: NL 16-byte chunks per thread for one K stage
// (NT threads; thread t owns chunk t % 8 of rows t / 8 + (NT / 8) i).
template <int NL, int NCH, int NT = 256>
__device__ __forceinline__ void gload(u32x4 (&r)[NL], const uint8_t* const (&p)[NL], uint32_t kt, uint32_t t) {
#pragma unroll
  for (int i = 0; i < NL; i++)
    if (NCH % NT == 0 || t + NT * i < (uint32_t)NCH)
      r[i] = *(g_u32x4*)(uintptr_t)(p[i] + kt * kRowBytes);
}

// Registers -> one LDS stage (swizzled rows).
template <int NL, int NCH, int NT = 256>
__device__ __forceinline__ void sstore(uint8_t* stage, const u32x4 (&r)[NL], uint32_t t, uint32_t chunk) {
#pragma unroll
  for (int i = 0; i < NL; i++)
    if (NCH % NT == 0 || t + NT * i < (uint32_t)NCH)
      *reinterpret_cast<u32x4*>(stage + swz((t >> 3) + (NT / 8) * i, chunk)) = r[i];
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

    store_tile<FM, FN>(acc, la, gr, m0 + wm * WM, n0 + wn * WN, relu, out_f32, lane);
  }
}


// ---------------------------------------------------------------------------
// Large-tile variant: BM x BN tile per workgroup of NT = 64 * waves threads,
// wave tile WM x WN.  Tiles are dealt to the 8 XCDs in contiguous ranges
// (workgroup w runs on XCD w % 8) of a tile list ordered by group, then by
// super-columns of SC n-tiles, m-tile fastest inside a super-column, so the
// workgroups that run together on one XCD share their A and W K-slices in
// that XCD's L2.
constexpr uint32_t kXcds = 8;

__device__ __forceinline__ void tile_coords(uint32_t local, uint32_t m_tiles, uint32_t n_tiles, uint32_t sc,
                                            uint32_t* mt, uint32_t* nt) {
  const uint32_t per_sc = m_tiles * sc;
  const uint32_t s = local / per_sc, r = local % per_sc;
  const uint32_t width = (s + 1) * sc <= n_tiles ? sc : n_tiles - s * sc;
  *mt = r / width;
  *nt = s * sc + r % width;
}

template <int BM, int BN, int WM, int WN>
__device__ __forceinline__ void ggemm2(const GemmHdr* __restrict__ hdr, const GemmGroup* __restrict__ groups,
                                       const LayerArgs la, uint8_t* lds) {
  constexpr int NWN = BN / WN, NWM = BM / WM;
  constexpr int NT = 64 * NWN * NWM;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int A_CH = BM * 8, B_CH = BN * 8;
  constexpr int A_LD = (A_CH + NT - 1) / NT, B_LD = (B_CH + NT - 1) / NT;
  constexpr uint32_t A_STAGE = BM * kRowBytes, B_STAGE = BN * kRowBytes;
  constexpr uint32_t SC = 4;
  uint8_t* const As = lds;
  uint8_t* const Bs = lds + 2 * A_STAGE;

  const uint32_t t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const uint32_t wm = wave / NWN, wn = wave % NWN;
  const uint32_t N = la.N, K = la.K;
  const uint32_t total = hdr->total_tiles, G = hdr->n_groups;
  const uint32_t ld_chunk = t & 7;
  const bool out_f32 = la.flags & kOutF32, relu = la.flags & kRelu;
  const uint32_t KT = K / BK;
  const uint32_t n_tiles = N / BN;

  // this workgroup's XCD range of the tile list
  const uint32_t xcd = blockIdx.x % kXcds, j = blockIdx.x / kXcds, per_xcd = gridDim.x / kXcds;
  if (j >= per_xcd) return;  // the host launches a multiple of 8 workgroups
  const uint32_t r0 = (uint32_t)(((uint64_t)total * xcd) / kXcds);
  const uint32_t r1 = (uint32_t)(((uint64_t)total * (xcd + 1)) / kXcds);

  for (uint32_t tile = r0 + j; tile < r1; tile += per_xcd) {
    const GemmGroup gr = groups[find_group(groups, G, tile)];
    const uint32_t m_tiles = (gr.m + BM - 1) / BM;
    uint32_t mt, nt;
    tile_coords(tile - gr.tile_start, m_tiles, n_tiles, SC, &mt, &nt);
    const uint32_t m0 = mt * BM, n0 = nt * BN;
    const uint64_t* wtab = reinterpret_cast<const uint64_t*>(gr.wtab);

    const uint8_t* ap[A_LD];
    const uint8_t* bp[B_LD];
#pragma unroll
    for (int i = 0; i < A_LD; i++) {
      const uint32_t row = (t >> 3) + (NT / 8) * i;
      uint32_t r = m0 + (row < BM ? row : 0);
      r = r < gr.m ? r : gr.m - 1;
      ap[i] = a_row(la, gr.row0 + r, 2) + ld_chunk * 16;
    }
#pragma unroll
    for (int i = 0; i < B_LD; i++) {
      const uint32_t row = (t >> 3) + (NT / 8) * i;
      const uint64_t off = la.w_off + (uint64_t)(n0 + (row < BN ? row : 0)) * K * 2;
      bp[i] = reinterpret_cast<const uint8_t*>(wtab[off >> kBlockShift]) + (off & (kBlock - 1)) + ld_chunk * 16;
    }

    f32x4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; i++)
#pragma unroll
      for (int jj = 0; jj < FN; jj++) acc[i][jj] = f32x4{0.f, 0.f, 0.f, 0.f};

    u32x4 ra[A_LD], rb[B_LD];
    gload<A_LD, A_CH, NT>(ra, ap, 0, t);
    gload<B_LD, B_CH, NT>(rb, bp, 0, t);
    sstore<A_LD, A_CH, NT>(As, ra, t, ld_chunk);
    sstore<B_LD, B_CH, NT>(Bs, rb, t, ld_chunk);
    __syncthreads();
    for (uint32_t kt = 0; kt < KT; kt++) {
      const uint32_t cur = kt & 1;
      if (kt + 1 < KT) {
        gload<A_LD, A_CH, NT>(ra, ap, kt + 1, t);
        gload<B_LD, B_CH, NT>(rb, bp, kt + 1, t);
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
        for (int jj = 0; jj < FN; jj++) {
          const uint32_t r = wn * WN + jj * 16 + (lane & 15);
          bfr[jj] = *reinterpret_cast<const bf16x8*>(Bs + cur * B_STAGE + swz(r, chunk));
        }
#pragma unroll
        for (int i = 0; i < FM; i++)
#pragma unroll
          for (int jj = 0; jj < FN; jj++)
            acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[jj], acc[i][jj], 0, 0, 0);
      }
      if (kt + 1 < KT) {
        sstore<A_LD, A_CH, NT>(As + (cur ^ 1) * A_STAGE, ra, t, ld_chunk);
        sstore<B_LD, B_CH, NT>(Bs + (cur ^ 1) * B_STAGE, rb, t, ld_chunk);
      }
      __syncthreads();
    }

    store_tile<FM, FN>(acc, la, gr, m0 + wm * WM, n0 + wn * WN, relu, out_f32, lane);
  }
}

// ---------------------------------------------------------------------------
// Direct-to-LDS variant: K stages of 32 (64 B per row) in an S-deep ring,
// filled by global_load_lds_dwordx4 (each wave instruction writes 1 KiB of
// LDS: 16 rows x 64 B; lane i lands at byte 16 i, so it fetches the global
// chunk that the swizzle puts there).  Loads for stage kt + S - 1 are issued
// right after the barrier of iteration kt, so S - 1 stages are in flight
// while one is computed.  Same MFMA and K order as the other shapes.
constexpr int kRow3 = 64;  // bytes of a row per stage (32 BF16)

// byte offset of chunk c (0..3) of row r in a [rows][32] stage; rows pair up
// in 128-byte bank lines, so the chunk is XOR-ed with (r / 2) mod 4.
__device__ __forceinline__ uint32_t swz3(uint32_t r, uint32_t c) { return r * kRow3 + ((c ^ ((r >> 1) & 3)) << 4); }

template <int N>
__device__ __forceinline__ void wait_vm() {
  // s_waitcnt vmcnt(N), expcnt and lgkmcnt left unconstrained
  __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// s_waitcnt until at most min(later, L) stages of LPS loads each are in flight
template <int LPS, int L>
__device__ __forceinline__ void wait_stages(uint32_t later) {
  if constexpr (L <= 0) {
    wait_vm<0>();
  } else {
    if (later >= (uint32_t)L) wait_vm<L * LPS>();
    else wait_stages<LPS, L - 1>(later);
  }
}

// S-slice ring of 32-wide K slices, consumed KG slices per barrier: a step
// waits for its KG slices, refills the KG ring positions the previous step
// read, then multiplies slice by slice (the K order of every other shape).
template <int BM, int BN, int WM, int WN, int S, int KG = 1>
__device__ __forceinline__ void ggemm3(const GemmHdr* __restrict__ hdr, const GemmGroup* __restrict__ groups,
                                       const LayerArgs la, uint8_t* lds) {
  constexpr int NWN = BN / WN, NWM = BM / WM;
  constexpr int NW = NWN * NWM, NT = 64 * NW;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr uint32_t A_STAGE = BM * kRow3, B_STAGE = BN * kRow3, STAGE = A_STAGE + B_STAGE;
  constexpr int A_INS = BM / 16 / NW, B_INS = BN / 16 / NW;  // 1 KiB load instructions per wave per stage
  static_assert(A_INS * 16 * NW == BM && B_INS * 16 * NW == BN, "rows split evenly over waves");
  constexpr int LPS = A_INS + B_INS;  // loads per wave per stage
  constexpr uint32_t SC = 4;
  typedef __attribute__((address_space(3))) void lds_void;

  const uint32_t t = threadIdx.x, lane = t & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const uint32_t wm = wave / NWN, wn = wave % NWN;
  const uint32_t N = la.N, K = la.K;
  const uint32_t total = hdr->total_tiles, G = hdr->n_groups;
  const bool out_f32 = la.flags & kOutF32, relu = la.flags & kRelu;
  const uint32_t KT = K / 32;
  const uint32_t n_tiles = N / BN;
  const uint32_t lrow = lane >> 2, lslot = lane & 3;

  const uint32_t xcd = blockIdx.x % kXcds, j = blockIdx.x / kXcds, per_xcd = gridDim.x / kXcds;
  if (j >= per_xcd) return;
  const uint32_t r0 = (uint32_t)(((uint64_t)total * xcd) / kXcds);
  const uint32_t r1 = (uint32_t)(((uint64_t)total * (xcd + 1)) / kXcds);

  for (uint32_t tile = r0 + j; tile < r1; tile += per_xcd) {
    const GemmGroup gr = groups[find_group(groups, G, tile)];
    const uint32_t m_tiles = (gr.m + BM - 1) / BM;
    uint32_t mt, nt;
    tile_coords(tile - gr.tile_start, m_tiles, n_tiles, SC, &mt, &nt);
    const uint32_t m0 = mt * BM, n0 = nt * BN;
    const uint64_t* wtab = reinterpret_cast<const uint64_t*>(gr.wtab);

    // per lane: the global chunk it fetches for each of the wave's load instructions
    const uint8_t* ap[A_INS];
    const uint8_t* bp[B_INS];
#pragma unroll
    for (int q = 0; q < A_INS; q++) {
      const uint32_t row = (wave * A_INS + q) * 16 + lrow;
      uint32_t r = m0 + row;
      r = r < gr.m ? r : gr.m - 1;
      const uint32_t chunk = lslot ^ ((row >> 1) & 3);
      ap[q] = a_row(la, gr.row0 + r, 2) + chunk * 16;
    }
#pragma unroll
    for (int q = 0; q < B_INS; q++) {
      const uint32_t row = (wave * B_INS + q) * 16 + lrow;
      const uint64_t off = la.w_off + (uint64_t)(n0 + row) * K * 2;
      const uint32_t chunk = lslot ^ ((row >> 1) & 3);
      bp[q] = reinterpret_cast<const uint8_t*>(wtab[off >> kBlockShift]) + (off & (kBlock - 1)) + chunk * 16;
    }
    auto issue = [&](uint32_t kt) __attribute__((always_inline)) {
      uint8_t* st = lds + (kt % S) * STAGE;
#pragma unroll
      for (int q = 0; q < A_INS; q++)
        __builtin_amdgcn_global_load_lds((const void*)(ap[q] + kt * kRow3),
                                         (lds_void*)(st + (wave * A_INS + q) * 1024), 16, 0, 0);
#pragma unroll
      for (int q = 0; q < B_INS; q++)
        __builtin_amdgcn_global_load_lds((const void*)(bp[q] + kt * kRow3),
                                         (lds_void*)(st + A_STAGE + (wave * B_INS + q) * 1024), 16, 0, 0);
    };

    f32x4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; i++)
#pragma unroll
      for (int jj = 0; jj < FN; jj++) acc[i][jj] = f32x4{0.f, 0.f, 0.f, 0.f};

    static_assert(S >= 2 * KG, "a step refills only positions the previous step read");
#pragma unroll
    for (int s0 = 0; s0 < S - KG; s0++)
      if ((uint32_t)s0 < KT) issue(s0);
    for (uint32_t kt0 = 0; kt0 < KT; kt0 += KG) {
      // slices issued after this step's last one: min(S - 2 KG, KT - kt0 - KG)
      const uint32_t later = (KT - kt0 - KG) < (uint32_t)(S - 2 * KG) ? (KT - kt0 - KG) : (uint32_t)(S - 2 * KG);
      wait_stages<LPS, S - 2 * KG>(later);
      // plain barrier: the wait above already covers this wave's loads
      __builtin_amdgcn_s_barrier();
#pragma unroll
      for (int g = 0; g < KG; g++)
        if (kt0 + S - KG + g < KT) issue(kt0 + S - KG + g);
#pragma unroll
      for (int g = 0; g < KG; g++) {
        const uint8_t* st = lds + ((kt0 + g) % S) * STAGE;
        const uint32_t chunk = lane >> 4;
        bf16x8 af[FM], bfr[FN];
#pragma unroll
        for (int i = 0; i < FM; i++) {
          const uint32_t r = wm * WM + i * 16 + (lane & 15);
          af[i] = *reinterpret_cast<const bf16x8*>(st + swz3(r, chunk));
        }
#pragma unroll
        for (int jj = 0; jj < FN; jj++) {
          const uint32_t r = wn * WN + jj * 16 + (lane & 15);
          bfr[jj] = *reinterpret_cast<const bf16x8*>(st + A_STAGE + swz3(r, chunk));
        }
#pragma unroll
        for (int i = 0; i < FM; i++)
#pragma unroll
          for (int jj = 0; jj < FN; jj++)
            acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[jj], acc[i][jj], 0, 0, 0);
      }
    }
    __syncthreads();  // the next tile's first loads overwrite stages still being read

    store_tile<FM, FN>(acc, la, gr, m0 + wm * WM, n0 + wn * WN, relu, out_f32, lane);
  }
}

// ---------------------------------------------------------------------------
// Ping-pong schedule over the ggemm3 ring: the waves form two groups of
// equal size (waves w and w + NW / 2 share a SIMD; 8 waves: groups of four).
// Every wave alternates a memory phase (LDS reads of one K-slice's
// fragments, global loads of a later slice) and a matrix phase (that slice's
// MFMAs), each ended by a workgroup barrier;
// the second group starts one barrier late, so while one wave of a SIMD
// multiplies, its partner fetches.  Ring safety: a slice's buffer is
// refilled S - 1 slices later, after both groups' reads of it completed
// (lgkmcnt(0) before each phase's barrier); a slice is read only after
// every wave waited for its own loads of it before an earlier barrier.
__device__ __forceinline__ void phase_sync() {
  __builtin_amdgcn_sched_barrier(0);
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_sched_barrier(0);
}

template <int BM, int BN, int WM, int WN, int S, bool PRIO = false>
__device__ __forceinline__ void ggemm6(const GemmHdr* __restrict__ hdr, const GemmGroup* __restrict__ groups,
                                       const LayerArgs la, uint8_t* lds) {
  constexpr int NWN = BN / WN, NWM = BM / WM;
  constexpr int NW = NWN * NWM;
  static_assert(NW % 8 == 0, "two groups, each with the same number of waves on every SIMD");
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr uint32_t A_STAGE = BM * kRow3, B_STAGE = BN * kRow3, STAGE = A_STAGE + B_STAGE;
  constexpr int A_INS = BM / 16 / NW, B_INS = BN / 16 / NW;
  static_assert(A_INS * 16 * NW == BM && B_INS * 16 * NW == BN, "rows split evenly over waves");
  constexpr int LPS = A_INS + B_INS;
  constexpr uint32_t SC = 4;
  typedef __attribute__((address_space(3))) void lds_void;

  const uint32_t t = threadIdx.x, lane = t & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const uint32_t wm = wave / NWN, wn = wave % NWN;
  const bool lag = wave >= NW / 2;  // waves w and w + NW / 2 share a SIMD
  const uint32_t N = la.N, K = la.K;
  const uint32_t total = hdr->total_tiles, G = hdr->n_groups;
  const bool out_f32 = la.flags & kOutF32, relu = la.flags & kRelu;
  const uint32_t KT = K / 32;
  const uint32_t n_tiles = N / BN;
  const uint32_t lrow = lane >> 2, lslot = lane & 3;

  const uint32_t xcd = blockIdx.x % kXcds, j = blockIdx.x / kXcds, per_xcd = gridDim.x / kXcds;
  if (j >= per_xcd) return;
  const uint32_t r0 = (uint32_t)(((uint64_t)total * xcd) / kXcds);
  const uint32_t r1 = (uint32_t)(((uint64_t)total * (xcd + 1)) / kXcds);

  for (uint32_t tile = r0 + j; tile < r1; tile += per_xcd) {
    const GemmGroup gr = groups[find_group(groups, G, tile)];
    const uint32_t m_tiles = (gr.m + BM - 1) / BM;
    uint32_t mt, nt;
    tile_coords(tile - gr.tile_start, m_tiles, n_tiles, SC, &mt, &nt);
    const uint32_t m0 = mt * BM, n0 = nt * BN;
    const uint64_t* wtab = reinterpret_cast<const uint64_t*>(gr.wtab);

    const uint8_t* ap[A_INS];
    const uint8_t* bp[B_INS];
#pragma unroll
    for (int q = 0; q < A_INS; q++) {
      const uint32_t row = (wave * A_INS + q) * 16 + lrow;
      uint32_t r = m0 + row;
      r = r < gr.m ? r : gr.m - 1;
      ap[q] = a_row(la, gr.row0 + r, 2) + (lslot ^ ((row >> 1) & 3)) * 16;
    }
#pragma unroll
    for (int q = 0; q < B_INS; q++) {
      const uint32_t row = (wave * B_INS + q) * 16 + lrow;
      const uint64_t off = la.w_off + (uint64_t)(n0 + row) * K * 2;
      bp[q] = reinterpret_cast<const uint8_t*>(wtab[off >> kBlockShift]) + (off & (kBlock - 1)) +
              (lslot ^ ((row >> 1) & 3)) * 16;
    }
    auto issue = [&](uint32_t kt) __attribute__((always_inline)) {
      uint8_t* st = lds + (kt % S) * STAGE;
#pragma unroll
      for (int q = 0; q < A_INS; q++)
        __builtin_amdgcn_global_load_lds((const void*)(ap[q] + kt * kRow3),
                                         (lds_void*)(st + (wave * A_INS + q) * 1024), 16, 0, 0);
#pragma unroll
      for (int q = 0; q < B_INS; q++)
        __builtin_amdgcn_global_load_lds((const void*)(bp[q] + kt * kRow3),
                                         (lds_void*)(st + A_STAGE + (wave * B_INS + q) * 1024), 16, 0, 0);
    };

    f32x4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; i++)
#pragma unroll
      for (int jj = 0; jj < FN; jj++) acc[i][jj] = f32x4{0.f, 0.f, 0.f, 0.f};

#pragma unroll
    for (int s0 = 0; s0 < S - 1; s0++)
      if ((uint32_t)s0 < KT) issue(s0);
    wait_stages<LPS, S - 2>((KT - 1) < (uint32_t)(S - 2) ? (KT - 1) : (uint32_t)(S - 2));
    phase_sync();  // slice 0 is in LDS
    if (lag) phase_sync();
    const uint32_t chunk = lane >> 4;
    for (uint32_t kt = 0; kt < KT; kt++) {
      // memory phase
      const uint8_t* st = lds + (kt % S) * STAGE;
      bf16x8 af[FM], bfr[FN];
#pragma unroll
      for (int i = 0; i < FM; i++)
        af[i] = *reinterpret_cast<const bf16x8*>(st + swz3(wm * WM + i * 16 + (lane & 15), chunk));
#pragma unroll
      for (int jj = 0; jj < FN; jj++)
        bfr[jj] = *reinterpret_cast<const bf16x8*>(st + A_STAGE + swz3(wn * WN + jj * 16 + (lane & 15), chunk));
      if (kt + S - 1 < KT) issue(kt + S - 1);
      if (kt + 1 < KT) {
        const uint32_t later = (KT - 2 - kt) < (uint32_t)(S - 2) ? (KT - 2 - kt) : (uint32_t)(S - 2);
        wait_stages<LPS, S - 2>(later);  // this wave's loads of slice kt + 1 landed
      }
      __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): fragments in registers, slice kt free
      phase_sync();
      // matrix phase
      if (PRIO) __builtin_amdgcn_s_setprio(1);
#pragma unroll
      for (int i = 0; i < FM; i++)
#pragma unroll
        for (int jj = 0; jj < FN; jj++)
          acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[jj], acc[i][jj], 0, 0, 0);
      if (PRIO) __builtin_amdgcn_s_setprio(0);
      phase_sync();
    }
    if (!lag) phase_sync();  // both groups leave the tile after the same number of barriers

    store_tile<FM, FN>(acc, la, gr, m0 + wm * WM, n0 + wn * WN, relu, out_f32, lane);
  }
}

}  // namespace

#define SAGE_GGEMM(BM, BN, WM, WN, OCC)                                                               \
  extern "C" __global__ __launch_bounds__(256, OCC) void ggemm_bf16_##BM##x##BN(                       \
      const GemmHdr* __restrict__ hdr, const GemmGroup* __restrict__ groups, LayerArgs la) {           \
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * (BM + BN) * kRowBytes];                    \
    ggemm_bf16<BM, BN, WM, WN>(hdr, groups, la, lds);                                                  \
  }

SAGE_GGEMM(32, 128, 32, 32, 2)
SAGE_GGEMM(64, 128, 32, 64, 2)
SAGE_GGEMM(128, 128, 64, 64, 2)

// large tiles, 8 waves, XCD-aware tile ranges
#define SAGE_GGEMM2(BM, BN, WM, WN)                                                                   \
  extern "C" __global__ __launch_bounds__(64 * (BM / WM) * (BN / WN), 1) void ggemm2_bf16_##BM##x##BN(  \
      const GemmHdr* __restrict__ hdr, const GemmGroup* __restrict__ groups, LayerArgs la) {           \
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * (BM + BN) * kRowBytes];                    \
    ggemm2<BM, BN, WM, WN>(hdr, groups, la, lds);                                                      \
  }

SAGE_GGEMM2(128, 256, 64, 64)

// direct-to-LDS, S-stage ring
#define SAGE_GGEMM3G(NAME, BM, BN, WM, WN, S, G)                                                      \
  extern "C" __global__ __launch_bounds__(64 * (BM / WM) * (BN / WN), 1) void NAME(                    \
      const GemmHdr* __restrict__ hdr, const GemmGroup* __restrict__ groups, LayerArgs la) {           \
    __shared__ __attribute__((aligned(1024))) uint8_t lds[S * (BM + BN) * kRow3];                      \
    ggemm3<BM, BN, WM, WN, S, G>(hdr, groups, la, lds);                                                \
  }
#define SAGE_GGEMM3(NAME, BM, BN, WM, WN, S) SAGE_GGEMM3G(NAME, BM, BN, WM, WN, S, 1)
// thin tiles with an eight-stage ring: a few rows (small batches, and the
// ragged last row tiles split off a large-tile launch) are bound by the
// latency of the K walk, which the deep ring hides
SAGE_GGEMM3(ggemm3_bf16_128x64, 128, 64, 32, 64, 8)
// sixteen-slice rings consumed four slices per barrier (K a multiple of 128)
SAGE_GGEMM3G(ggemm3g4_bf16_16x64, 16, 64, 16, 64, 16, 4)
SAGE_GGEMM3G(ggemm3g4_bf16_32x64, 32, 64, 16, 64, 16, 4)
SAGE_GGEMM3G(ggemm3g4_bf16_64x64, 64, 64, 32, 32, 16, 4)
// narrow thin tiles: a few rows still spread W over 128..256 workgroups
// (16 x 16 with its register use capped at two waves per SIMD)
#define SAGE_GGEMM3T(NAME, BM, BN, WM, WN, S, G, WPE)                                                 \
  extern "C" __global__ __launch_bounds__(64 * (BM / WM) * (BN / WN))                                  \
      __attribute__((amdgpu_waves_per_eu(WPE))) void NAME(                                             \
      const GemmHdr* __restrict__ hdr, const GemmGroup* __restrict__ groups, LayerArgs la) {           \
    __shared__ __attribute__((aligned(1024))) uint8_t lds[S * (BM + BN) * kRow3];                      \
    ggemm3<BM, BN, WM, WN, S, G>(hdr, groups, la, lds);                                                \
  }
SAGE_GGEMM3T(ggemm3t_bf16_16x16, 16, 16, 16, 16, 16, 4, 2)
SAGE_GGEMM3G(ggemm3t_bf16_16x32, 16, 32, 16, 32, 16, 4)
SAGE_GGEMM3G(ggemm3t_bf16_32x32, 32, 32, 16, 32, 16, 4)

// ping-pong over the direct-to-LDS ring
#define SAGE_GGEMM6(NAME, BM, BN, WM, WN, S, PRIO)                                                    \
  extern "C" __global__ __launch_bounds__(64 * (BM / WM) * (BN / WN), 1) void NAME(                    \
      const GemmHdr* __restrict__ hdr, const GemmGroup* __restrict__ groups, LayerArgs la) {           \
    __shared__ __attribute__((aligned(1024))) uint8_t lds[S * (BM + BN) * kRow3];                      \
    ggemm6<BM, BN, WM, WN, S, PRIO>(hdr, groups, la, lds);                                             \
  }
// the matrix-phase wave at raised issue priority
SAGE_GGEMM6(ggemm6p_bf16_256x256, 256, 256, 128, 64, 4, true)
SAGE_GGEMM6(ggemm6_bf16_256x128, 256, 128, 64, 64, 4, false)

// ---------------------------------------------------------------- FP32 MLP
// A few rows are bound by load latency, not bandwidth: every load of a
// K chunk goes out before the first FMA, straight into registers.
constexpr uint32_t kF32KC = 2048;                       // K per chunk
typedef __attribute__((address_space(1))) const f32x4 g_f32x4;

// The value of lane l ^ m (m a power of two below 64) for every lane of the
// wave.  Within a row of 16 lanes through DPP: m = 1, 2 by quad permutation,
// 8 by a rotation of the row by 8, 4 by rotations by 4 and 12 (a lane with
// bit 2 set takes the one that reads 4 lanes down, i.e. lane l - 4); 16 and
// 32 through the LDS crossbar.  Every lane of the wave must execute it.
__device__ __forceinline__ float lane_xor(float x, int m, uint32_t lane) {
  const int xi = __builtin_bit_cast(int, x);
  int r;
  if (m == 1) r = __builtin_amdgcn_mov_dpp(xi, 0xB1, 0xF, 0xF, false);        // quad_perm [1,0,3,2]
  else if (m == 2) r = __builtin_amdgcn_mov_dpp(xi, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
  else if (m == 8) r = __builtin_amdgcn_mov_dpp(xi, 0x128, 0xF, 0xF, false);  // row_ror:8
  else if (m == 4) {
    const int down = __builtin_amdgcn_mov_dpp(xi, 0x124, 0xF, 0xF, false);  // row_ror:4: lane l reads l - 4
    const int up = __builtin_amdgcn_mov_dpp(xi, 0x12C, 0xF, 0xF, false);    // row_ror:12: lane l reads l + 4
    r = (lane & 4) ? down : up;
  } else {
    return __shfl_xor(x, m, 64);
  }
  return __builtin_bit_cast(float, r);
}

// K split over the waves.  Tiles: (group, block of CW output columns); the
// four waves of the workgroup share the tile's CW columns and split each
// 2048-wide K chunk into quarters: wave w takes k in [kc + w kn/4, kc +
// (w + 1) kn/4), lane l the float4 at 4l and 4l + 256 of that quarter.  Every
// lane loads its slice of the 8 input rows and of the CW weight rows straight
// into registers (no staging, no barrier before the FMAs) and accumulates 8 x
// CW partial sums with fmaf in k order.  The lanes' sums are combined by a
// halving exchange (partners l ^ 1, l ^ 2, l ^ 8, l ^ 4, l ^ 16, l ^ 32: each
// step a lane keeps half of its values and adds its partner's copy of that
// half), the waves' in LDS in wave order.  The order depends only on K,
// not on the rows of the launch.
template <int CW, bool ONE>
__device__ __forceinline__ void mlp_f32_ks_body(const GemmHdr* __restrict__ hdr, const GemmGroup* __restrict__ groups,
                                                const LayerArgs& la, float (*red)[8 * CW], const uint64_t* wtab1,
                                                uint32_t m1) {
  static_assert(CW == 4 || CW == 8, "4 or 8 columns per workgroup");
  constexpr int V = 8 * CW;  // partial sums per lane: 8 rows x CW columns
  const uint32_t t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const uint32_t K = la.K;
  const bool relu = la.flags & kRelu;
  const uint32_t total_tiles = ONE ? la.N / CW : hdr->total_tiles;
  for (uint32_t tile = blockIdx.x; tile < total_tiles; tile += gridDim.x) {
    GemmGroup gr;
    if (ONE) gr = GemmGroup{reinterpret_cast<uint64_t>(wtab1), m1, 0, 0, 0};
    else gr = groups[find_group(groups, hdr->n_groups, tile)];
    const uint32_t n = (tile - gr.tile_start) * CW;
    const uint64_t* wtab = reinterpret_cast<const uint64_t*>(gr.wtab);
    // the block-table entries of the CW weight rows: every load issued
    // before the first is used (one round trip, not CW)
    uint64_t went[CW];
#pragma unroll
    for (int c = 0; c < CW; c++) went[c] = wtab[(la.w_off + (uint64_t)(n + c) * K * 4) >> kBlockShift];
    const float* wr[CW];
#pragma unroll
    for (int c = 0; c < CW; c++)
      wr[c] = reinterpret_cast<const float*>(went[c] + ((la.w_off + (uint64_t)(n + c) * K * 4) & (kBlock - 1)));
    for (uint32_t r0 = 0; r0 < gr.m; r0 += 8) {
      const uint32_t nr = gr.m - r0 < 8 ? gr.m - r0 : 8;
      // rows past the group's end read its first row of the block (not
      // stored); row-table entries, like the block-table ones, all go out
      // before the first is used
      const float* ar[8];
      if (la.a_tab) {
        uint64_t rent[8];
#pragma unroll
        for (int i = 0; i < 8; i++) rent[i] = la.a_tab[gr.row0 + r0 + ((uint32_t)i < nr ? i : 0)];
#pragma unroll
        for (int i = 0; i < 8; i++) ar[i] = reinterpret_cast<const float*>(rent[i]);
      } else {
#pragma unroll
        for (int i = 0; i < 8; i++)
          ar[i] = reinterpret_cast<const float*>(la.a_base +
                                                 (uint64_t)(gr.row0 + r0 + ((uint32_t)i < nr ? i : 0)) * K * 4);
      }
      float acc[8][CW];
#pragma unroll
      for (int i = 0; i < 8; i++)
#pragma unroll
        for (int c = 0; c < CW; c++) acc[i][c] = 0.f;
      for (uint32_t kc = 0; kc < K; kc += kF32KC) {
        const uint32_t kn = K - kc < kF32KC ? K - kc : kF32KC;  // a power of two >= 128
        const uint32_t kw = kn / 4, base = kc + wave * kw;
        f32x4 xv[8][2], wv[CW][2];
#pragma unroll
        for (int j = 0; j < 2; j++) {
          const uint32_t k4 = 4 * (lane + 64 * j);
          const uint32_t k = base + (k4 < kw ? k4 : 0);  // idle lanes of a narrow chunk load in bounds
#pragma unroll
          for (int c = 0; c < CW; c++) wv[c][j] = *(g_f32x4*)(uintptr_t)(wr[c] + k);
#pragma unroll
          for (int i = 0; i < 8; i++) xv[i][j] = *(g_f32x4*)(uintptr_t)(ar[i] + k);
        }
#pragma unroll
        for (int j = 0; j < 2; j++) {
          if (4 * (lane + 64 * j) < kw) {
#pragma unroll
            for (int i = 0; i < 8; i++)
#pragma unroll
              for (int c = 0; c < CW; c++) {
                acc[i][c] = fmaf(xv[i][j].x, wv[c][j].x, acc[i][c]);
                acc[i][c] = fmaf(xv[i][j].y, wv[c][j].y, acc[i][c]);
                acc[i][c] = fmaf(xv[i][j].z, wv[c][j].z, acc[i][c]);
                acc[i][c] = fmaf(xv[i][j].w, wv[c][j].w, acc[i][c]);
              }
          }
        }
      }
      // halving exchange: at the step with lane mask m a lane keeps half of its
      // values (the upper half if its bit m is set) and adds its partner's
      // (lane l ^ m) copy of that half, so each kept value becomes the sum over
      // twice as many lanes.  Masks 1, 2, 8, 4 (DPP within a row of 16), then
      // 16 and 32 (through LDS) on the few values left; V = 32 ends with a
      // plain exchange over mask 32.  The value a lane ends with is read off
      // its bits: the bit of each step's mask picks the half it kept.
      float v[V];
#pragma unroll
      for (int i = 0; i < 8; i++)
#pragma unroll
        for (int c = 0; c < CW; c++) v[i * CW + c] = acc[i][c];
      constexpr int kMask[6] = {1, 2, 8, 4, 16, 32};
      uint32_t idx = 0;
#pragma unroll
      for (int st = 0, h = V / 2; h >= 1; st++, h >>= 1) {
        const int m = kMask[st];
        const bool up = lane & m;
        if (up) idx += h;
#pragma unroll
        for (int q = 0; q < h; q++) {
          const float keep = up ? v[q + h] : v[q], send = up ? v[q] : v[q + h];
          v[q] = keep + lane_xor(send, m, lane);
        }
      }
      if constexpr (V == 32) v[0] += lane_xor(v[0], 32, lane);
      if (V == 64 || (lane & 32) == 0) red[wave][idx] = v[0];
      __syncthreads();
      if (t < (uint32_t)V) {
        const uint32_t i = t / CW, c = t % CW;
        if (i < nr) {
          float s = red[0][t] + red[1][t];
          s += red[2][t];
          s += red[3][t];
          if (relu) s = s > 0.f ? s : 0.f;
          reinterpret_cast<float*>(c_row(la, gr.row0 + r0 + i, 4))[n + c] = s;
        }
      }
      __syncthreads();  // the next row block reuses red
    }
  }
}

#define SAGE_F32KS(NAME, CW)                                                                            \
  extern "C" __global__ __launch_bounds__(256) void NAME(const GemmHdr* __restrict__ hdr,                \
                                                         const GemmGroup* __restrict__ groups,           \
                                                         LayerArgs la, const uint64_t* wtab1, uint32_t m1) { \
    __shared__ float red[4][8 * CW];                                                                     \
    if (wtab1) mlp_f32_ks_body<CW, true>(hdr, groups, la, red, wtab1, m1);                               \
    else mlp_f32_ks_body<CW, false>(hdr, groups, la, red, wtab1, m1);                                    \
  }
// ONE: the launch has a single group, passed by value (its block table
// `wtab1` and row count `m1`, row0 and first tile 0): the header and group
// record are not read, which takes two dependent loads off the way to the
// weights.
SAGE_F32KS(mlp_f32_layer, 4)
SAGE_F32KS(mlp_f32_layer_c8, 8)
