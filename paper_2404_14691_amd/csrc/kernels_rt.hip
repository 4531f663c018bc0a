// Runtime kernels of the data-preparation path, built into libsage.so:
//   fp64k   - FP64K-v1 fingerprint of every 64 KiB block of a device buffer
//   blkcopy - per-block COPY into pool slots, or byte-for-byte VERIFY
// Both are HBM-streaming kernels: 16-byte coalesced loads, all of a block's
// loads issued before any use, one workgroup per block (grid-stride).
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace sage {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Keyed product of one 64-bit word j: ((lo + a_j) mod 2^32) * ((hi + c_j) mod 2^32).
__device__ __forceinline__ uint64_t nh_term(uint32_t lo, uint32_t hi, uint32_t a, uint32_t c) {
  return (uint64_t)(lo + a) * (uint64_t)(hi + c);
}

// 256 threads per block.  Thread t reads the 16-byte pieces i*4096 + 16t
// (i < 16), i.e. words j = 512i + 2t and 512i + 2t + 1, so its keys advance
// by 512*K1 / 512*K3 per piece.  The sum is commutative mod 2^64, so the
// wave shuffle + LDS reduction order does not change the result.
__global__ __launch_bounds__(256) void fp64k_kernel(const uint8_t* __restrict__ data, uint64_t nbytes,
                                                    uint64_t* __restrict__ out, uint32_t nblocks) {
  __shared__ uint64_t red[4];
  const uint32_t t = threadIdx.x;
  const uint64_t nfull = nbytes >> kBlockShift;
  const uint32_t a0 = kFpK0 + (2u * t) * kFpK1;
  const uint32_t c0 = kFpK2 + (2u * t) * kFpK3;
  const uint32_t a_step = 512u * kFpK1, c_step = 512u * kFpK3;
  for (uint32_t b = blockIdx.x; b < nblocks; b += gridDim.x) {
    uint64_t acc = 0;
    const uint8_t* base = data + ((uint64_t)b << kBlockShift);
    uint64_t L;
    if (b < nfull) {
      L = kBlock;
      const u32x4* p = reinterpret_cast<const u32x4*>(base) + t;
      u32x4 v[16];
#pragma unroll
      for (int i = 0; i < 16; i++) v[i] = __builtin_nontemporal_load(p + i * 256);
      uint32_t a = a0, c = c0;
#pragma unroll
      for (int i = 0; i < 16; i++) {
        acc += nh_term(v[i].x, v[i].y, a, c);
        acc += nh_term(v[i].z, v[i].w, a + kFpK1, c + kFpK3);
        a += a_step;
        c += c_step;
      }
    } else {
      // short last block: word by word, zero-padded to 8 bytes
      L = nbytes - ((uint64_t)b << kBlockShift);
      const uint32_t nw = (uint32_t)((L + 7) >> 3);
      for (uint32_t j = t; j < nw; j += 256) {
        uint64_t w = 0;
        if (8ull * (j + 1) <= L) {
          w = *reinterpret_cast<const uint64_t*>(base + 8ull * j);
        } else {
          for (uint32_t q = 0; 8ull * j + q < L; q++) w |= (uint64_t)base[8ull * j + q] << (8 * q);
        }
        acc += nh_term((uint32_t)w, (uint32_t)(w >> 32), kFpK0 + j * kFpK1, kFpK2 + j * kFpK3);
      }
    }
    acc = wave_sum_u64(acc);
    if ((t & 63) == 0) red[t >> 6] = acc;
    __syncthreads();
    if (t == 0) {
      const uint64_t s = red[0] + red[1] + red[2] + red[3];
      out[b] = mix64(s ^ (L * kFpK4));
    }
    __syncthreads();
  }
}

// One block operation by one workgroup: COPY moves len bytes, VERIFY
// compares them (result = 1 when any byte differs).  Full blocks move as
// 16 x 16 B per thread with all loads first; short blocks use a strided
// loop plus single bytes.
__device__ __forceinline__ void block_op(const BlkOp& op, uint32_t* result, uint32_t t) {
  const u32x4* s = reinterpret_cast<const u32x4*>(op.src);
  const uint32_t nvec = op.len >> 4;
  if (op.op == 0) {
    u32x4* d = reinterpret_cast<u32x4*>(op.dst);
    if (nvec == kBlock / 16) {
      u32x4 v[16];
#pragma unroll
      for (int i = 0; i < 16; i++) v[i] = __builtin_nontemporal_load(s + t + i * 256);
#pragma unroll
      for (int i = 0; i < 16; i++) __builtin_nontemporal_store(v[i], d + t + i * 256);
    } else {
      for (uint32_t i = t; i < nvec; i += 256) d[i] = s[i];
      const uint32_t q = nvec * 16 + t;
      if (q < op.len) reinterpret_cast<uint8_t*>(op.dst)[q] = reinterpret_cast<const uint8_t*>(op.src)[q];
    }
  } else {
    const u32x4* d = reinterpret_cast<const u32x4*>(op.dst);
    int diff = 0;
    if (nvec == kBlock / 16) {
      u32x4 v[8], w[8];
#pragma unroll
      for (int h = 0; h < 2; h++) {
#pragma unroll
        for (int i = 0; i < 8; i++) {
          v[i] = __builtin_nontemporal_load(s + t + (h * 8 + i) * 256);
          w[i] = __builtin_nontemporal_load(d + t + (h * 8 + i) * 256);
        }
#pragma unroll
        for (int i = 0; i < 8; i++)
          diff |= (v[i].x != w[i].x) | (v[i].y != w[i].y) | (v[i].z != w[i].z) | (v[i].w != w[i].w);
      }
    } else {
      for (uint32_t i = t; i < nvec; i += 256) {
        const u32x4 a = s[i], b = d[i];
        diff |= (a.x != b.x) | (a.y != b.y) | (a.z != b.z) | (a.w != b.w);
      }
      const uint32_t q = nvec * 16 + t;
      if (q < op.len)
        diff |= reinterpret_cast<const uint8_t*>(op.src)[q] != reinterpret_cast<const uint8_t*>(op.dst)[q];
    }
    diff = __syncthreads_or(diff);
    if (t == 0) *result = diff ? 1u : 0u;
  }
}

// Two operations per workgroup iteration: when both are full-block COPYs
// all 32 loads of the pair are in flight before the first store
// (nontemporal both ways: the data is not read again soon).  For launches
// of more blocks than one wave of workgroups holds.
__global__ __launch_bounds__(256) void blkcopy_kernel(const BlkOp* __restrict__ ops, uint32_t n,
                                                      uint32_t* __restrict__ result) {
  const uint32_t t = threadIdx.x;
  for (uint32_t o = blockIdx.x * 2u; o < n; o += gridDim.x * 2u) {
    const BlkOp op0 = ops[o];
    const bool has1 = o + 1 < n;
    const BlkOp op1 = has1 ? ops[o + 1] : op0;
    if (has1 && op0.op == 0 && op1.op == 0 && op0.len == kBlock && op1.len == kBlock) {
      const u32x4* s0 = reinterpret_cast<const u32x4*>(op0.src);
      const u32x4* s1 = reinterpret_cast<const u32x4*>(op1.src);
      u32x4* d0 = reinterpret_cast<u32x4*>(op0.dst);
      u32x4* d1 = reinterpret_cast<u32x4*>(op1.dst);
      u32x4 v[32];
#pragma unroll
      for (int i = 0; i < 16; i++) {
        v[i] = __builtin_nontemporal_load(s0 + t + i * 256);
        v[16 + i] = __builtin_nontemporal_load(s1 + t + i * 256);
      }
#pragma unroll
      for (int i = 0; i < 16; i++) {
        __builtin_nontemporal_store(v[i], d0 + t + i * 256);
        __builtin_nontemporal_store(v[16 + i], d1 + t + i * 256);
      }
    } else {
      block_op(op0, result + o, t);
      if (has1) block_op(op1, result + o + 1, t);
    }
  }
}

// One operation per workgroup, for launches that fit in one wave of
// workgroups (the registration path's 1228-4096 blocks): single blocks
// balance such a wave across the CUs better than pairs (3-4 % less time
// per launch at 1228-8192 scattered blocks, HIP events per launch).
__global__ __launch_bounds__(256) void blkcopy1_kernel(const BlkOp* __restrict__ ops, uint32_t n,
                                                       uint32_t* __restrict__ result) {
  const uint32_t o = blockIdx.x;
  if (o < n) block_op(ops[o], result + o, threadIdx.x);
}

// Measurement kernel, not on the path: the grouped BF16 GEMM's main tile
// shape (256 x 256, 8 waves, wave tile 128 x 64, v_mfma_f32_16x16x32_bf16
// over K slices of 32, two wave groups alternating LDS and matrix phases at
// raised matrix-phase priority) with its global loads taken out.  The
// four-stage LDS ring (64 B of each of 512 rows per stage, the same swizzle)
// is filled once with random BF16 values of activation and weight scale, and
// every slice reads its fragments from the next stage, so operand values
// change from slice to slice as in a real layer (the MFMA rate and the
// clock the chip sustains depend on them).  Its time bounds what the main
// shape reaches on this chip with this data.  Each workgroup also records
// its shader-clock and 100 MHz reference-clock counts, whose ratio is that
// clock.
typedef __bf16 ceil_bf16x8 __attribute__((ext_vector_type(8)));
typedef float ceil_f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void ceil_sync() {
  __builtin_amdgcn_sched_barrier(0);
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_sched_barrier(0);
}

// a random BF16: random sign and 7-bit fraction, exponent in [e0, e0 + 7)
__device__ __forceinline__ uint32_t ceil_bf16(uint32_t h, uint32_t e0) {
  return ((h >> 31) << 15) | ((e0 + (h >> 8) % 7u) << 7) | (h & 0x7Fu);
}

__global__ __launch_bounds__(512, 1) void mfma_ceiling_kernel(uint32_t k_slices, float* __restrict__ out,
                                                             unsigned long long* __restrict__ clk) {
  constexpr uint32_t kRow = 64, kStage = 512 * kRow, kAStage = 256 * kRow;
  __shared__ __attribute__((aligned(1024))) uint8_t lds[4 * kStage];
  const uint32_t t = threadIdx.x, lane = t & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const uint32_t wm = wave / 4, wn = wave % 4;
  const bool lag = wave >= 4;  // waves w and w + 4 share a SIMD
  for (uint32_t w = t; w < 4 * kStage / 4; w += 512) {
    uint32_t h = (w + 1) * 0x9E3779B9u ^ blockIdx.x * 0x85EBCA6Bu;
    h ^= h >> 16;
    h *= 0x7FEB352Du;
    h ^= h >> 15;
    h *= 0x846CA68Bu;
    h ^= h >> 16;
    const uint32_t e0 = (w * 4) % kStage < kAStage ? 120u : 114u;  // A rows ~[2^-7, 1), W rows 64 x smaller
    reinterpret_cast<uint32_t*>(lds)[w] = ceil_bf16(h, e0) | (ceil_bf16(h * 0x27D4EB2Du, e0) << 16);
  }
  __syncthreads();
  auto sw = [](uint32_t r, uint32_t c) { return r * kRow + ((c ^ ((r >> 1) & 3)) << 4); };
  ceil_f32x4 acc[8][4];
#pragma unroll
  for (int i = 0; i < 8; i++)
#pragma unroll
    for (int j = 0; j < 4; j++) acc[i][j] = ceil_f32x4{0.f, 0.f, 0.f, 0.f};
  const unsigned long long c0 = __builtin_amdgcn_s_memtime(), r0 = __builtin_amdgcn_s_memrealtime();
  ceil_sync();
  if (lag) ceil_sync();
  const uint32_t chunk = lane >> 4;
  for (uint32_t kt = 0; kt < k_slices; kt++) {
    const uint8_t* st = lds + (kt % 4) * kStage;
    ceil_bf16x8 af[8], bfr[4];
#pragma unroll
    for (int i = 0; i < 8; i++) af[i] = *reinterpret_cast<const ceil_bf16x8*>(st + sw(wm * 128 + i * 16 + (lane & 15), chunk));
#pragma unroll
    for (int j = 0; j < 4; j++)
      bfr[j] = *reinterpret_cast<const ceil_bf16x8*>(st + kAStage + sw(wn * 64 + j * 16 + (lane & 15), chunk));
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
    ceil_sync();
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int i = 0; i < 8; i++)
#pragma unroll
      for (int j = 0; j < 4; j++) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    __builtin_amdgcn_s_setprio(0);
    ceil_sync();
  }
  if (!lag) ceil_sync();
  float sum = 0.f;
#pragma unroll
  for (int i = 0; i < 8; i++)
#pragma unroll
    for (int j = 0; j < 4; j++) sum += acc[i][j][0] + acc[i][j][1] + acc[i][j][2] + acc[i][j][3];
  out[blockIdx.x * 512u + t] = sum;
  if (t == 0) {
    clk[2 * blockIdx.x] = __builtin_amdgcn_s_memtime() - c0;
    clk[2 * blockIdx.x + 1] = __builtin_amdgcn_s_memrealtime() - r0;
  }
}

// Scratch of fn_invoke_noalloc (metadata + activations), a fixed array in
// every GPU's copy of this code object.  Host code never passes `scratch`
// itself (on the host it is only a stand-in symbol): it passes the device
// address that noalloc_scratch looked up for the current device.
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(int device, uint8_t** out) {
  static std::mutex mu;
  static uint8_t* addr[64] = {};
  if (device < 0 || device >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[device] = static_cast<uint8_t*>(p);
  }
  *out = addr[device];
  return hipSuccess;
}

hipError_t launch_fp64k(const void* data, uint64_t nbytes, uint64_t* out, int max_groups, hipStream_t s) {
  if (nbytes == 0) return hipSuccess;
  const uint32_t nblocks = (uint32_t)((nbytes + kBlock - 1) >> kBlockShift);
  const uint32_t grid = nblocks < (uint32_t)max_groups ? nblocks : (uint32_t)max_groups;
  hipLaunchKernelGGL(fp64k_kernel, dim3(grid), dim3(256), 0, s, static_cast<const uint8_t*>(data), nbytes, out,
                     nblocks);
  return hipGetLastError();
}

hipError_t launch_blkcopy(const BlkOp* ops, uint32_t n, uint32_t* result, int max_groups, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (n <= (uint32_t)max_groups) {
    hipLaunchKernelGGL(blkcopy1_kernel, dim3(n), dim3(256), 0, s, ops, n, result);
  } else {
    const uint32_t pairs = (n + 1) / 2;
    const uint32_t grid = pairs < (uint32_t)max_groups ? pairs : (uint32_t)max_groups;
    hipLaunchKernelGGL(blkcopy_kernel, dim3(grid), dim3(256), 0, s, ops, n, result);
  }
  return hipGetLastError();
}

hipError_t launch_mfma_ceiling(uint32_t grid, uint32_t k_slices, float* out, unsigned long long* clk, hipStream_t s) {
  hipLaunchKernelGGL(mfma_ceiling_kernel, dim3(grid), dim3(512), 0, s, k_slices, out, clk);
  return hipGetLastError();
}

}  // namespace sage
