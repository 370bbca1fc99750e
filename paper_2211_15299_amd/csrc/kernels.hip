// HIP kernels (gfx950) of the homogeneous-support DFT.
//
// Data layout and index conventions shared by the kernels
// ---------------------------------------------------------
// A transform of size k = 2^S works on an array X[0..k) of complex64.  The
// input arrives in ascending order of the sample set I_r: position a holds
// f(i_p) with p = bitrev_S(a), where p is the position of the same sample in
// the recursion order of the pivoted sampling pattern (Sec. VII).  The radix-2
// recursion of Lemma 3 is an iterative decimation-in-time over p; expressed
// over a it pairs, at stage u (pivot r_u, u = 1..S), the positions a and
// a + 2^{S-u}, and the butterfly
//     X[a] <- P + w Q,   X[a + 2^{S-u}] <- P - w Q   (P = X[a], Q = X[a+2^{S-u}])
// uses the twiddle of node q_lo = bitrev_{u-1}(a >> (S-u+1)).  After S stages
// position a holds (k/N) (Ff)(j) for the j with q(j) = bitrev_S(a).
//
// Twiddle table (device, "a-order"): entry (2^{u-1} - 1) + h holds the twiddle
// of stage u and node q_lo = bitrev_{u-1}(h), so a thread that knows the top
// u-1 bits h of its position reads its twiddle without a bit reversal and
// neighbouring lanes read neighbouring entries.  k - 1 entries in all.
//
// Output table src[t] = bitrev_S(q(J[t])): the array position holding the
// coefficient of J[t], for a coalesced gather-and-store in the caller's order.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <atomic>

#include "launch.h"

namespace hidft {

// ---------------------------------------------------------------------------
// Twiddle generation: exp(-i pi m / 2^d) evaluated in FP64, rounded once.
// ---------------------------------------------------------------------------
__global__ void twiddle_gen_kernel(const uint64_t* __restrict__ num,
                                   const uint8_t* __restrict__ log2den,
                                   float2* __restrict__ out, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // x = m / 2^d is in [0, 1); exact whenever m < 2^53.
  const double x = ldexp((double)num[i], -(int)log2den[i]);
  double sn, cs;
  sincospi(x, &sn, &cs);
  out[i] = make_float2((float)cs, (float)(-sn));
}

hipError_t launch_twiddle_gen(const uint64_t* d_num, const uint8_t* d_den, float2* d_tw,
                              uint64_t n, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const unsigned threads = 256;
  const unsigned blocks = (unsigned)((n + threads - 1) / threads);
  hipLaunchKernelGGL(twiddle_gen_kernel, dim3(blocks), dim3(threads), 0, stream, d_num,
                     d_den, d_tw, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Butterfly: (P, Q) <- (P + w Q, P - w Q) in six FMAs.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void butterfly(float2& P, float2& Q, const float2 w) {
  float xr = fmaf(w.x, Q.x, P.x);
  xr = fmaf(-w.y, Q.y, xr);
  float xi = fmaf(w.x, Q.y, P.y);
  xi = fmaf(w.y, Q.x, xi);
  Q.x = fmaf(2.0f, P.x, -xr);
  Q.y = fmaf(2.0f, P.y, -xi);
  P.x = xr;
  P.y = xi;
}

// Workgroup barrier that orders LDS accesses only.  __syncthreads() also
// orders global memory, which makes every wave wait for its outstanding
// global stores (the previous signal's outputs) before the barrier; the
// exchanges here only need the LDS writes of the block to be visible.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Wave priority (s_setprio, an issue-arbitration hint among the waves of a
// SIMD; it changes no result): a wave runs at priority 2 while it issues a
// signal's sample loads and at 1 while it gathers and stores the
// coefficients, and at 0 during the transform, so the memory requests of
// one block go out ahead of the other blocks' arithmetic.  Measured: 2^12
// points 50.0 -> 48.7 us, 2^14 points 66.1 -> 63.5 us, the inverse map at
// 2^12 points 51.7 -> 50.7 us; 2^13 unchanged.  The grouped launch (slower
// with it) and the Shift-and-Sample loads (unchanged) do not use it.
//
// Occupancy of a kernel: blocks resident per CU and the CU count, queried
// once per kernel (the first call also raises its dynamic LDS limit).
struct Occupancy {
  int per_cu = 0;
  int cus = 0;
};

// A kernel's occupancy, queried on the first call from any thread.  per_cu
// is stored before cus (release); a reader that sees cus != 0 (acquire) also
// sees per_cu and the LDS limit the query raised.  Threads racing on the
// first call each run the query and store the same values.
struct OccupancyCache {
  std::atomic<int> per_cu{0}, cus{0};
  bool get(Occupancy* o) const {
    const int c = cus.load(std::memory_order_acquire);
    if (c == 0) return false;
    o->cus = c;
    o->per_cu = per_cu.load(std::memory_order_relaxed);
    return true;
  }
  void put(const Occupancy& o) {
    per_cu.store(o.per_cu, std::memory_order_relaxed);
    cus.store(o.cus, std::memory_order_release);
  }
};

static hipError_t query_occupancy(const void* kernel, int threads, size_t lds_bytes,
                                  Occupancy* occ) {
  hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds_bytes);
  if (e != hipSuccess) return e;
  int dev = 0, cus = 0, per_cu = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) !=
      hipSuccess)
    return e;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds_bytes)) !=
      hipSuccess)
    return e;
  occ->per_cu = per_cu > 0 ? per_cu : 1;
  occ->cus = cus > 0 ? cus : 1;
  return hipSuccess;
}

// Samples and coefficients are read or written exactly once: their loads and
// stores carry the non-temporal cache policy (measured: about 7% less time
// than cached stores at 2^12 points), while the plan tables, which every
// signal reuses, stay cached.
typedef float f2v_t __attribute__((ext_vector_type(2)));
constexpr int CPOL_NT = 2;  // cache-policy operand of the buffer builtins: nt

__device__ __forceinline__ float2 load_stream(const float2* p) {
  return __builtin_bit_cast(float2, __builtin_nontemporal_load(reinterpret_cast<const f2v_t*>(p)));
}
__device__ __forceinline__ void store_stream(float2* p, float2 x) {
  __builtin_nontemporal_store(__builtin_bit_cast(f2v_t, x), reinterpret_cast<f2v_t*>(p));
}

// LDS padding: one spare slot after every 2^RHO complex values keeps the
// strided accesses of the radix-2^RHO groups spread over the 64 LDS banks.
template <int RHO>
__device__ __forceinline__ int lds_pad(int a) { return a + (a >> RHO); }

// The padded slot of base + (c << lo) for a group window [lo, lo + RHO):
// with base = a_lo + (a_hi << (lo + RHO)), a_lo < 2^lo, and c < 2^RHO the low
// lo + RHO bits never carry, so
//   lds_pad(base + (c << lo)) = lds_pad(base) + (c << lo) + (c >> (RHO - lo))
// for lo < RHO, and + (c << (lo - RHO)) for lo >= RHO.  The per-c part is a
// compile-time constant (an LDS instruction offset), the rest one add per
// thread and group.
template <int RHO>
__device__ __forceinline__ constexpr int lds_window_off(int c, int lo) {
  return (c << lo) + (lo >= RHO ? (c << (lo - RHO)) : (c >> (RHO - lo)));
}

// The padded slot of c * T + tau for T a multiple of 2^RHO: lds_pad(tau) plus
// a per-c constant.
template <int RHO>
__device__ __forceinline__ constexpr int lds_column_off(int c, int T) {
  return c * T + ((c * T) >> RHO);
}

template <int S, int SCHED = SCHED_SHORT_FIRST, int RH = 4>
struct FusedShape {
  static constexpr int RHO = S < RH ? S : RH;                    // log2 points per thread
  static constexpr int R = 1 << RHO;
  static constexpr int K = 1 << S;
  static constexpr int T = K / R;                                // threads per signal
  static constexpr int SPB = T >= 256 ? 1 : 256 / T;             // signals per block
  static constexpr int THREADS = T * SPB;
  static constexpr int G = S == 0 ? 0 : (S + RHO - 1) / RHO;     // radix groups
  // Stages of group 1.  When RHO does not divide S one group is short:
  // SHORT_FIRST makes it group 1 (run straight from the global load),
  // SHORT_LAST makes group 1 a full radix-2^RHO group and the last one short.
  static constexpr int G1 = S == 0 ? 0
                            : (SCHED == SCHED_SHORT_LAST && S >= RHO) ? RHO
                                                                      : S - (G - 1) * RHO;
  // Group g >= 2 runs the stages of bits [lo(g), hi(g)) of a.  Its threads
  // always hold the RHO bits [lo(g), lo(g) + RHO): a short last group also
  // carries bits of the previous group, on which it runs no stage, and starts
  // at stage t0(g) of the window.
  static constexpr int hi(int g) { return S - G1 - (g - 2) * RHO; }
  static constexpr int lo(int g) { return hi(g) > RHO ? hi(g) - RHO : 0; }
  static constexpr int t0(int g) { return RHO - (hi(g) - lo(g)); }
  static constexpr int PADK = K + (K >> RHO);                    // LDS slots per signal
  static constexpr size_t LDS_BYTES = (size_t)SPB * PADK * sizeof(float2);
  // Launch strategy.  Up to 2^12 points the grid is persistent (blocks
  // resident per CU times the CU count) and walks over the batch: the
  // twiddles of groups 2..G and the gather positions a thread needs are
  // loaded once per block and kept in registers, and the next signals'
  // samples are loaded while the current ones are transformed.  Above (BIG:
  // 512 or 1024 threads and 68 or 136 KB of LDS per signal, at most 128
  // registers per thread) the tables do not fit in registers; read per signal,
  // their loads would queue behind a prefetch (vector memory counters retire
  // in order), so BIG sizes run one signal per block with a grid of one block
  // per signal.
  static constexpr bool BIG = S >= 14 || (S == 13 && RH == 5);
  static constexpr bool TW_REGS = !BIG && (G - 1) * (R - 1) <= 45;
  static constexpr int NTW = G > 1 ? (TW_REGS ? (G - 1) * (R - 1) : 1) : 1;
};

// One thread's values of a signal.
template <int S, int RH>
using SigVec = float2[FusedShape<S, SCHED_SHORT_FIRST, RH>::R];

// ---------------------------------------------------------------------------
// Group 1 on the matrix cores (PREC_F16X2, PREC_BF16X3).
//
// The four stages of a full group 1 multiply every column of 16 values
// (a = col + c T, c < 16, col < T = 2^{S-4}) by the same 16 x 16 complex
// matrix W, the product of the four butterfly stages; its entries have unit
// modulus.  As a real product, Re(Wx) = [Re W, -Im W] [Re x; Im x] and
// Im(Wx) = [Im W, Re W] [Re x; Im x]: two 16 x 32 by 32 x 16 MFMA products
// (v_mfma_f32_16x16x32_{f16,bf16}) per tile of 16 columns, FP32 accumulation.
//
// Operand layout: lane l holds row or column l & 15 and the 8 consecutive
// k-entries 8 (l >> 4) .. + 7, here the interleaved (re, im) pairs of
// c = 4 (l >> 4) .. + 3; the result holds rows 4 (l >> 4) .. + 3 of column
// l & 15.  So lane l of wave w keeps, for tile j < 4, the values c = 4 (l >> 4)
// + i (i < 4) of block column 64 w + 16 j + (l & 15) before and after the
// product.
//
// Radix 32 (k >= 2^13, short group last): the five stages of group 1 form a
// 32 x 32 matrix, applied as 2 x 2 blocks of 16 x 16 (four times the
// products).  A lane then keeps, per tile, the values c = 16 kc + 4 (l >> 4)
// + i of both 16-value halves kc of its column.
//
// Split precision: x = x1 + x2 (+ x3) and W = W1 + W2 (+ W3) in FP16 (two
// terms) or BF16 (three terms); the products of the leading terms are summed
// in FP32, smallest first.
//   F16X2:  x W ~ W1 x1 + W1 x2 + W2 x1.  FP16 has a narrow exponent range, so
//           each column is first scaled by a power of two that brings its
//           largest component into [2^14, 2^15) (exact; undone after).
//   BF16X3: x W ~ W1 x1 + W1 x2 + W2 x1 + W1 x3 + W2 x2 + W3 x1, no scaling.
// The split operands of W are computed in FP64 on the device at plan creation
// (stage_matrix_kernel).
// ---------------------------------------------------------------------------
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// Offsets (in 16-byte operands) of the split operands in a plan's table.
constexpr int AMAT_F16_OPS = 4;   // Re-row hi, lo; Im-row hi, lo
constexpr int AMAT_BF16_OPS = 6;  // Re-row terms 1..3; Im-row terms 1..3
constexpr int AMAT_BF16_BASE = AMAT_F16_OPS * 64;

// Operand set of the group-1 matrix: NB = 1 block (radix 16) or NB = 4 blocks
// b = 2 rb + kc (radix 32).
template <int PREC, int NB = 1>
struct MfmaOps {};
template <int NB>
struct MfmaOps<PREC_F16X2, NB> {
  half8_t rh[NB], rl[NB], ih[NB], il[NB];
};
template <int NB>
struct MfmaOps<PREC_BF16X3, NB> {
  bf16x8_t r1[NB], r2[NB], r3[NB], i1[NB], i2[NB], i3[NB];
};

// Blocks of the operand set for groups of RHO stages.
template <int RHO>
constexpr int mfma_blocks() { return RHO == 5 ? 4 : 1; }

// The radix-32 operands follow the radix-16 ones in a plan's table.
template <int PREC, int NB>
__device__ __forceinline__ MfmaOps<PREC, NB> load_mfma_ops(const uint4* __restrict__ amat) {
  MfmaOps<PREC, NB> op;
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const uint4* a = amat + (NB == 4 ? 1 + b : 0) * (AMAT_BYTES / 16);
    if constexpr (PREC == PREC_F16X2) {
      op.rh[b] = __builtin_bit_cast(half8_t, a[0 * 64 + l]);
      op.rl[b] = __builtin_bit_cast(half8_t, a[1 * 64 + l]);
      op.ih[b] = __builtin_bit_cast(half8_t, a[2 * 64 + l]);
      op.il[b] = __builtin_bit_cast(half8_t, a[3 * 64 + l]);
    } else if constexpr (PREC == PREC_BF16X3) {
      const uint4* q = a + AMAT_BF16_BASE;
      op.r1[b] = __builtin_bit_cast(bf16x8_t, q[0 * 64 + l]);
      op.r2[b] = __builtin_bit_cast(bf16x8_t, q[1 * 64 + l]);
      op.r3[b] = __builtin_bit_cast(bf16x8_t, q[2 * 64 + l]);
      op.i1[b] = __builtin_bit_cast(bf16x8_t, q[3 * 64 + l]);
      op.i2[b] = __builtin_bit_cast(bf16x8_t, q[4 * 64 + l]);
      op.i3[b] = __builtin_bit_cast(bf16x8_t, q[5 * 64 + l]);
    }
  }
  return op;
}

// Group 1 of the 64 block columns of this wave (v in the MFMA layout).  Per
// tile of 16 columns a lane holds NV = R / 4 values: for radix 32 the column's
// 32 values are two k-chunks kc of 16 (inputs) and two row blocks rb of 16
// (outputs), and W is multiplied block by block, (rb, kc) = operand block
// 2 rb + kc.  The products are summed smallest term first over both chunks.
template <int PREC, int R>
__device__ __forceinline__ void group1_mfma(float2 (&v)[R],
                                            const MfmaOps<PREC, (R == 32 ? 4 : 1)>& op) {
  static_assert(R == 16 || R == 32, "radix-16 or radix-32 group 1");
  constexpr int NV = R / 4;   // values per lane and tile
  constexpr int NK = R / 16;  // input chunks = output row blocks
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float2* x = v + NV * j;
    if constexpr (PREC == PREC_F16X2) {
      float mx = 0.f;
#pragma unroll
      for (int i = 0; i < NV; ++i) mx = fmaxf(mx, fmaxf(fabsf(x[i].x), fabsf(x[i].y)));
      // The column's values sit in lanes l, l ^ 16, l ^ 32, l ^ 48.
      mx = fmaxf(mx, __shfl_xor(mx, 16));
      mx = fmaxf(mx, __shfl_xor(mx, 32));
      int e = (int)((__builtin_bit_cast(uint32_t, mx) >> 23) & 0xffu);
      e = e < 15 ? 15 : (e > 254 ? 254 : e);
      const float sc = __builtin_bit_cast(float, (uint32_t)(268 - e) << 23);   // 2^(141-e)
      const float inv = __builtin_bit_cast(float, (uint32_t)(e - 14) << 23);   // 2^(e-141)
      half8_t x1[NK], x2[NK];
#pragma unroll
      for (int kc = 0; kc < NK; ++kc) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const float xr = x[4 * kc + p].x * sc, xi = x[4 * kc + p].y * sc;
          const _Float16 hr = (_Float16)xr, hi = (_Float16)xi;
          x1[kc][2 * p] = hr;
          x1[kc][2 * p + 1] = hi;
          x2[kc][2 * p] = (_Float16)(xr - (float)hr);
          x2[kc][2 * p + 1] = (_Float16)(xi - (float)hi);
        }
      }
#pragma unroll
      for (int rb = 0; rb < NK; ++rb) {
        float4_t dr = {0.f, 0.f, 0.f, 0.f}, di = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < NK; ++kc) {
          const int bk = NK == 2 ? 2 * rb + kc : 0;
          dr = __builtin_amdgcn_mfma_f32_16x16x32_f16(op.rl[bk], x1[kc], dr, 0, 0, 0);
          di = __builtin_amdgcn_mfma_f32_16x16x32_f16(op.il[bk], x1[kc], di, 0, 0, 0);
        }
#pragma unroll
        for (int kc = 0; kc < NK; ++kc) {
          const int bk = NK == 2 ? 2 * rb + kc : 0;
          dr = __builtin_amdgcn_mfma_f32_16x16x32_f16(op.rh[bk], x2[kc], dr, 0, 0, 0);
          di = __builtin_amdgcn_mfma_f32_16x16x32_f16(op.ih[bk], x2[kc], di, 0, 0, 0);
        }
#pragma unroll
        for (int kc = 0; kc < NK; ++kc) {
          const int bk = NK == 2 ? 2 * rb + kc : 0;
          dr = __builtin_amdgcn_mfma_f32_16x16x32_f16(op.rh[bk], x1[kc], dr, 0, 0, 0);
          di = __builtin_amdgcn_mfma_f32_16x16x32_f16(op.ih[bk], x1[kc], di, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) x[4 * rb + i] = make_float2(dr[i] * inv, di[i] * inv);
      }
    } else {
      bf16x8_t x1[NK], x2[NK], x3[NK];
#pragma unroll
      for (int kc = 0; kc < NK; ++kc) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const float xv = q ? x[4 * kc + p].y : x[4 * kc + p].x;
            const __bf16 b1 = (__bf16)xv;
            const float r1 = xv - (float)b1;
            const __bf16 b2 = (__bf16)r1;
            const float r2 = r1 - (float)b2;
            x1[kc][2 * p + q] = b1;
            x2[kc][2 * p + q] = b2;
            x3[kc][2 * p + q] = (__bf16)r2;
          }
        }
      }
#pragma unroll
      for (int rb = 0; rb < NK; ++rb) {
        float4_t dr = {0.f, 0.f, 0.f, 0.f}, di = {0.f, 0.f, 0.f, 0.f};
        // Term pairs (W term, x term), smallest first: (1,3) (2,2) (3,1) (1,2) (2,1) (1,1).
#define HIDFT_BF16_TERM(WR, WI, X)                                                 \
  _Pragma("unroll") for (int kc = 0; kc < NK; ++kc) {                              \
    const int bk = NK == 2 ? 2 * rb + kc : 0;                                      \
    dr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(op.WR[bk], X[kc], dr, 0, 0, 0);    \
    di = __builtin_amdgcn_mfma_f32_16x16x32_bf16(op.WI[bk], X[kc], di, 0, 0, 0);    \
  }
        HIDFT_BF16_TERM(r1, i1, x3)
        HIDFT_BF16_TERM(r2, i2, x2)
        HIDFT_BF16_TERM(r3, i3, x1)
        HIDFT_BF16_TERM(r1, i1, x2)
        HIDFT_BF16_TERM(r2, i2, x1)
        HIDFT_BF16_TERM(r1, i1, x1)
#undef HIDFT_BF16_TERM
#pragma unroll
        for (int i = 0; i < 4; ++i) x[4 * rb + i] = make_float2(dr[i], di[i]);
      }
    }
  }
}

// Split operands of the group-1 matrix W (2^RHO x 2^RHO, the product of
// stages 1..RHO, a-order twiddle entries 0..2^RHO - 2) in FP64, one wavefront
// per 16 x 16 block of W: block b = 2 rb + kc holds rows 16 rb .. 16 rb + 15
// and columns 16 kc .. 16 kc + 15 (radix 16: the single block b = 0).  Lane
// l = 16 g + m' builds W[m][c] for m = 16 rb + m' and c = 16 kc + 4 g + p
// (p < 4), then splits its row operands.
//
// The butterflies of the group connect input c to output m by exactly one
// path: stage u (bit b = RHO - u) moves the value from bit b of c to bit b of
// m, and multiplies it by 1 if bit b of c is 0, else by +w or -w (bit b of m
// 0 or 1), w the twiddle of the node named by the bits of m above b.  So
// W[m][c] is the product of those factors, in stage order.
template <int RHO>
__global__ void __launch_bounds__(64)
stage_matrix_kernel(const uint64_t* __restrict__ num, const uint8_t* __restrict__ log2den,
                    uint4* __restrict__ amat) {
  const int l = threadIdx.x;
  const int rb = blockIdx.x >> 1, kc = blockIdx.x & 1;
  const int g = l >> 4, m = 16 * rb + (l & 15);
  double Wr[4], Wi[4];
  for (int p = 0; p < 4; ++p) {
    const int c = 16 * kc + 4 * g + p;
    double xr = 1.0, xi = 0.0;
    for (int u = 1; u <= RHO; ++u) {
      const int bit = RHO - u;
      if (!((c >> bit) & 1)) continue;
      const int e = (1 << (u - 1)) - 1 + (m >> (bit + 1));
      double sn, cs;
      sincospi(ldexp((double)num[e], -(int)log2den[e]), &sn, &cs);
      const double wr = cs, wi = -sn;
      const double qr = wr * xr - wi * xi;
      const double qi = wr * xi + wi * xr;
      const bool neg = (m >> bit) & 1;
      xr = neg ? -qr : qr;
      xi = neg ? -qi : qi;
    }
    Wr[p] = xr;
    Wi[p] = xi;
  }
  // Row operands: element e pairs with (re, im)[e & 1] of column 16 kc + 4g + e/2.
  half8_t f16[4];
  bf16x8_t b16[6];
  for (int e = 0; e < 8; ++e) {
    const int p = e >> 1;
    const double ar = (e & 1) ? -Wi[p] : Wr[p];  // Re row: [Re W, -Im W]
    const double ai = (e & 1) ? Wr[p] : Wi[p];   // Im row: [Im W,  Re W]
    const double a[2] = {ar, ai};
    for (int q = 0; q < 2; ++q) {
      const _Float16 h = (_Float16)(float)a[q];
      f16[2 * q][e] = h;
      f16[2 * q + 1][e] = (_Float16)(float)(a[q] - (double)(float)h);
      const __bf16 b1 = (__bf16)(float)a[q];
      const double r1 = a[q] - (double)(float)b1;
      const __bf16 b2 = (__bf16)(float)r1;
      const double r2 = r1 - (double)(float)b2;
      b16[3 * q][e] = b1;
      b16[3 * q + 1][e] = b2;
      b16[3 * q + 2][e] = (__bf16)(float)r2;
    }
  }
  uint4* out = amat + blockIdx.x * (AMAT_BYTES / 16);
  for (int o = 0; o < AMAT_F16_OPS; ++o) out[o * 64 + l] = __builtin_bit_cast(uint4, f16[o]);
  for (int o = 0; o < AMAT_BF16_OPS; ++o)
    out[AMAT_BF16_BASE + o * 64 + l] = __builtin_bit_cast(uint4, b16[o]);
}

hipError_t launch_stage_matrix(const uint64_t* d_num, const uint8_t* d_den, void* d_amat,
                               bool radix32, hipStream_t stream) {
  uint4* am = static_cast<uint4*>(d_amat);
  hipLaunchKernelGGL(stage_matrix_kernel<4>, dim3(1), dim3(64), 0, stream, d_num, d_den, am);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !radix32) return e;
  hipLaunchKernelGGL(stage_matrix_kernel<5>, dim3(4), dim3(64), 0, stream, d_num, d_den,
                     am + AMAT_BYTES / 16);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fused batched transform.  Each block owns SPB signal slots of T threads.
// Per signal:
//   * group 1 (stages 1..G1, the top G1 bits of a) runs straight from the
//     global load: thread tau holds a = tau + c*T for c < R, so each load
//     instruction of a wavefront reads 64 consecutive samples (with MFMA,
//     16-sample runs, see above);
//   * every later group takes up to RHO = 4 stages (radix 16) on the next
//     lower bits of a, through LDS; each thread reads and writes back its own
//     16 slots, so one barrier per group suffices;
//   * the block gathers the outputs in the caller's order of J (src table),
//     scales by N/k and stores them coalesced.
// Up to 2^12 points the grid is persistent (blocks resident per CU times the
// CU count) and walks over the batch; the twiddles and gather positions a
// thread needs are then loaded once per block and kept in registers, and
// the next signals' samples are loaded while the current ones are
// transformed.  Larger sizes run one signal per block.
// ---------------------------------------------------------------------------
template <int S, int SCHED, int RH>
struct ThreadState {  // per-thread constants of the persistent form
  using Sh = FusedShape<S, SCHED, RH>;
  float2 w1[(1 << Sh::G1) > 1 ? (1 << Sh::G1) - 1 : 1];  // block-uniform (scalar registers)
  float2 wg[Sh::NTW];
  uint32_t srcpk[(Sh::R + 1) / 2];  // two 16-bit gather positions per register
};

// A value that is the same in every lane, moved to a scalar register.
__device__ __forceinline__ float2 make_uniform(float2 w) {
  w.x = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, w.x)));
  w.y = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, w.y)));
  return w;
}

// Access to one signal's tables and output row.  Every index is split into a
// part that is the same for all lanes (compile-time constants here) and a
// per-lane part.
//   FlatMem: plain global pointers.
//   BufMem:  buffer descriptors (base and size in scalar registers) with the
//            lane part as the one vector offset and the uniform part as a
//            scalar offset; it needs the signal to span whole wavefronts
//            (T >= 64) so that its descriptors are uniform.
// PARTIAL: only the first n_out outputs of the gather order are stored (the
// Shift-and-Sample workspace and direct paths); otherwise all of them, with
// no per-store predicate.
template <bool PARTIAL>
struct FlatMemT {
  const float2* tw;
  const uint16_t* src;
  float2* out;
  uint32_t n_out;
  __device__ __forceinline__ float2 tw_at(int uni, int lane) const { return tw[uni + lane]; }
  __device__ __forceinline__ int src_at(int uni, int lane) const { return src[uni + lane]; }
  __device__ __forceinline__ void put(int uni, int lane, float2 x) const {
    if constexpr (PARTIAL) {
      if ((uint32_t)(uni + lane) < n_out) store_stream(out + uni + lane, x);
    } else {
      store_stream(out + uni + lane, x);
    }
  }
};
using FlatMem = FlatMemT<false>;

// Twiddles of group g of the adjoint (stages t0(g)..RHO-1 of its window of
// bits) for the thread at lane tau: entry (1 << t) - 1 + h is the h-th of the
// window's stage t (entries of stages below t0(g) are left as they are).
template <int S, int SCHED, int N, class Mem>
__device__ __forceinline__ void adjoint_group_twiddles(float2 (&wq)[N], const Mem& mem, int tau,
                                                       int g) {
  using Sh = FusedShape<S, SCHED, 4>;
  constexpr int RHO = Sh::RHO;
  static_assert(N == (Sh::R > 1 ? Sh::R - 1 : 1), "one group's twiddles");
  const int lo = Sh::lo(g), t0 = Sh::t0(g);
  const int a_hi = tau >> lo;
#pragma unroll
  for (int t = 0; t < RHO; ++t) {
    if (t < t0) continue;
    const int u = S - lo - RHO + 1 + t;
#pragma unroll
    for (int h = 0; h < (1 << t); ++h)
      wq[(1 << t) - 1 + h] = mem.tw_at(((1 << (u - 1)) - 1) + h, a_hi << t);
  }
}

// Tables for the adjoint of one signal read per signal: its twiddles, the
// LDS places of the thread's R values (gather-table entries c * T + lane, the
// scatter that starts the adjoint) and the twiddles of its first group (the
// last group G of the forward order), both in registers.  They are read
// before the signal's values, so that the scatter and the first group do not
// wait for table reads queued behind the whole row (vector-memory counters
// retire in order).  The places ahead of the row took the adjoint passes of
// 2^15..2^21 points 4-5 us less per launch; the first group's twiddles
// ahead of it a further 1-1.4 us (3.8 us at 2^22), and the 2^14-point
// inverse (one signal per block) from 78 to 75 us.
template <int R, int T>
struct AdjointMem {
  static constexpr bool FIRST_TW = true;
  const float2* tw;
  int place[R];
  float2 first_tw[R > 1 ? R - 1 : 1];
  __device__ __forceinline__ void read_places(const uint16_t* src, int lane) {
#pragma unroll
    for (int c = 0; c < R; ++c) place[c] = src[c * T + lane];
  }
  template <int S, int SCHED>
  __device__ __forceinline__ void read_first_twiddles(int lane) {
    static_assert(FusedShape<S, SCHED, 4>::R == R && FusedShape<S, SCHED, 4>::T == T,
                  "the signal's shape");
#pragma unroll
    for (int i = 0; i < (R > 1 ? R - 1 : 1); ++i) first_tw[i] = make_float2(0.f, 0.f);
    adjoint_group_twiddles<S, SCHED>(first_tw, *this, lane, FusedShape<S, SCHED, 4>::G);
  }
  __device__ __forceinline__ float2 tw_at(int uni, int lane) const { return tw[uni + lane]; }
  __device__ __forceinline__ int src_at(int uni, int) const { return place[uni / T]; }
};
// Whether a table type holds its first group's twiddles (AdjointMem).
template <class M, class = void>
struct FirstTwOf {
  static constexpr bool value = false;
};
template <class M>
struct FirstTwOf<M, decltype((void)M::FIRST_TW)> {
  static constexpr bool value = M::FIRST_TW;
};

constexpr int BUFFER_DWORD3 = 0x00020000;  // raw buffer, 32-bit data format

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                          BUFFER_DWORD3);
}

struct BufMem {
  __amdgpu_buffer_rsrc_t tw, src, out;
  __device__ __forceinline__ float2 tw_at(int uni, int lane) const {
    return __builtin_bit_cast(float2,
                              __builtin_amdgcn_raw_buffer_load_b64(tw, lane * 8, uni * 8, 0));
  }
  __device__ __forceinline__ int src_at(int uni, int lane) const {
    return (int)__builtin_amdgcn_raw_buffer_load_b16(src, lane * 2, uni * 2, 0);
  }
  __device__ __forceinline__ void put(int uni, int lane, float2 x) const {
    __builtin_amdgcn_raw_buffer_store_b64(
        __builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, x), out, lane * 8,
        uni * 8, CPOL_NT);
  }
};

// R samples of one signal row for thread tau: v[c] = row[c*T + tau], through a
// buffer descriptor (BUF, the row must be wave-uniform) or a plain pointer.
template <int R, int T, bool BUF>
__device__ __forceinline__ void load_row(float2 (&v)[R], const float2* row, uint32_t k) {
  if constexpr (BUF) {
    static_assert(T >= 64, "a buffer descriptor needs a wave-uniform row");
    const __amdgpu_buffer_rsrc_t r = make_rsrc(row, k * 8u);
    const int tau = threadIdx.x & (T - 1);
#pragma unroll
    for (int c = 0; c < R; ++c)
      v[c] = __builtin_bit_cast(
          float2, __builtin_amdgcn_raw_buffer_load_b64(r, tau * 8, c * T * 8, CPOL_NT));
  } else {
    const int tau = threadIdx.x & (T - 1);
#pragma unroll
    for (int c = 0; c < R; ++c) v[c] = load_stream(row + c * T + tau);
  }
}

// Position of value e < 2^RHO / 4 of tile j of this thread in the MFMA layout
// (radix 2^RHO, RHO = 4 or 5): the block's signal slot and the position a
// within that signal.  The value is entry c = 16 (e >> 2) + 4 (lane >> 4) +
// (e & 3) of block column col.
template <int S, int RHO>
__device__ __forceinline__ void mfma_pos(int tid, int j, int e, int& slot, int& a) {
  constexpr int T = 1 << (S - RHO);  // columns per signal
  const int col = (tid & ~63) + 16 * j + (tid & 15);
  slot = col >> (S - RHO);
  a = (col & (T - 1)) + (16 * (e >> 2) + 4 * ((tid >> 4) & 3) + (e & 3)) * T;
}

// Loads the samples of the signals first_sig + slot (slot < SPB) that this
// thread holds for group 1: standard layout for FP32, MFMA layout otherwise.
// Signals at or beyond `batch` read as zeros.
template <int S, int SCHED, int RH, int PREC>
__device__ __forceinline__ void load_group1(SigVec<S, RH>& v, const float2* __restrict__ in,
                                            int64_t ld_in, uint64_t first_sig, uint64_t batch) {
  using Sh = FusedShape<S, SCHED, RH>;
  constexpr int R = Sh::R, T = Sh::T;
  const int tid = threadIdx.x;
  if constexpr (PREC == PREC_FP32) {
    const int slot = tid / T;
    const uint64_t sig = first_sig + slot;
    if (sig < batch) {
      load_row<R, T, false>(v, in + sig * (uint64_t)ld_in, 1u << S);
    } else {
#pragma unroll
      for (int c = 0; c < R; ++c) v[c] = make_float2(0.f, 0.f);
    }
  } else {
    constexpr int NV = R / 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
      for (int e = 0; e < NV; ++e) {
        int slot, a;
        mfma_pos<S, Sh::RHO>(tid, j, e, slot, a);
        const uint64_t sig = first_sig + slot;
        v[NV * j + e] =
            sig < batch ? load_stream(in + sig * (uint64_t)ld_in + a) : make_float2(0.f, 0.f);
      }
    }
  }
}

// Transform the samples in v (this thread's R values of group 1, in the
// layout of load_group1) and, if `store`, write the coefficients of this
// thread's signal slot through `mem`.  Lb is the block's LDS.  HOISTED:
// twiddles and gather positions come from `ts`, else from the tables behind
// `mem`.
// The block-wide barrier of transform_signal (every wave of the block takes
// part in each transform).
struct BlockSync {
  __device__ __forceinline__ void sync() { lds_barrier(); }
};

template <int S, int SCHED, int RH, int PREC, bool HOISTED, class Mem, class Sync = BlockSync>
__device__ __forceinline__ void transform_signal(SigVec<S, RH>& v, float2* Lb, int slot, int tau,
                                                 bool store, const Mem& mem, float scale,
                                                 const ThreadState<S, SCHED, RH>& ts,
                                                 const MfmaOps<PREC, mfma_blocks<RH>()>& op,
                                                 Sync sync = Sync()) {
  using Sh = FusedShape<S, SCHED, RH>;
  constexpr int RHO = Sh::RHO, R = Sh::R, T = Sh::T, G = Sh::G, G1 = Sh::G1;
  float2* L = Lb + slot * Sh::PADK;

  if constexpr (PREC == PREC_FP32) {
    // Group 1: stage u pairs bit RHO-u of c; the twiddle index is the top
    // u-1 bits of c, the same for every thread.
#pragma unroll
    for (int u = 1; u <= G1; ++u) {
      const int bit = RHO - u;
#pragma unroll
      for (int c = 0; c < R; ++c) {
        if (c & (1 << bit)) continue;
        const int idx = (1 << (u - 1)) - 1 + (c >> (bit + 1));
        butterfly(v[c], v[c | (1 << bit)], HOISTED ? ts.w1[idx] : mem.tw_at(idx, 0));
      }
    }
    if constexpr (T % R == 0) {
      const int pt = lds_pad<RHO>(tau);
#pragma unroll
      for (int c = 0; c < R; ++c) L[pt + lds_column_off<RHO>(c, T)] = v[c];
    } else {
#pragma unroll
      for (int c = 0; c < R; ++c) L[lds_pad<RHO>(c * T + tau)] = v[c];
    }
  } else {
    static_assert(S >= RHO && (RHO == 4 || RHO == 5) && G1 == RHO && RH == RHO,
                  "the matrix-core group 1 is a full radix-16 or radix-32 group");
    group1_mfma<PREC, R>(v, op);
    const int tid = threadIdx.x;
    constexpr int NV = R / 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
      for (int e = 0; e < NV; ++e) {
        int sl, a;
        mfma_pos<S, RHO>(tid, j, e, sl, a);
        Lb[sl * Sh::PADK + lds_pad<RHO>(a)] = v[NV * j + e];
      }
    }
  }

  // Groups 2..G on the window [lo, lo + RHO), stages t0..RHO-1 of it.
#pragma unroll
  for (int g = 2; g <= G; ++g) {
    const int lo = Sh::lo(g), t0 = Sh::t0(g);
    const int a_lo = tau & ((1 << lo) - 1);
    const int a_hi = tau >> lo;
    const int base = a_lo + (a_hi << (lo + RHO));
    // Without hoisted tables, the group's twiddles are requested before the
    // barrier, so that their latency overlaps the wait for the other waves.
    float2 wq[R > 1 ? R - 1 : 1];
    if constexpr (!(HOISTED && Sh::TW_REGS)) {
#pragma unroll
      for (int t = 0; t < RHO; ++t) {
        if (t < t0) continue;
        const int u = S - lo - RHO + 1 + t;
#pragma unroll
        for (int h = 0; h < (1 << t); ++h)
          wq[(1 << t) - 1 + h] = mem.tw_at(((1 << (u - 1)) - 1) + h, a_hi << t);
      }
    }
    sync.sync();
    const int pb = lds_pad<RHO>(base);
#pragma unroll
    for (int c = 0; c < R; ++c) v[c] = L[pb + lds_window_off<RHO>(c, lo)];
#pragma unroll
    for (int t = 0; t < RHO; ++t) {
      if (t < t0) continue;
      const int u = S - lo - RHO + 1 + t;
      const int bit = RHO - 1 - t;
#pragma unroll
      for (int c = 0; c < R; ++c) {
        if (c & (1 << bit)) continue;
        const int h = c >> (RHO - t);
        float2 w;
        if constexpr (HOISTED && Sh::TW_REGS)
          w = ts.wg[(g - 2) * (R - 1) + (1 << t) - 1 + h];
        else
          w = wq[(1 << t) - 1 + h];
        (void)u;
        butterfly(v[c], v[c | (1 << bit)], w);
      }
    }
#pragma unroll
    for (int c = 0; c < R; ++c) L[pb + lds_window_off<RHO>(c, lo)] = v[c];
  }
  // Gather positions of the output, requested before the last barrier.
  int pq[R];
  if constexpr (!HOISTED) {
    if (store) {
#pragma unroll
      for (int c = 0; c < R; ++c) pq[c] = mem.src_at(c * T, tau);
    }
  }
  sync.sync();

  // Wave priority 1 for the gather and stores (note on wave priority above).
  __builtin_amdgcn_s_setprio(1);
  if (store) {
#pragma unroll
    for (int c = 0; c < R; ++c) {
      const int p = HOISTED ? (int)((ts.srcpk[c >> 1] >> (16 * (c & 1))) & 0xffffu) : pq[c];
      const float2 x = L[lds_pad<RHO>(p)];
      mem.put(c * T, tau, make_float2(x.x * scale, x.y * scale));
    }
  }
  __builtin_amdgcn_s_setprio(0);
}

// Loads the per-thread constants: group-1 twiddles (uniform), the twiddles
// of groups 2..G this thread uses, and its gather positions.
template <int S, int SCHED, int RH, int PREC>
__device__ __forceinline__ void load_thread_state(ThreadState<S, SCHED, RH>& ts,
                                                  const float2* __restrict__ tw,
                                                  const uint16_t* __restrict__ src, int tau) {
  using Sh = FusedShape<S, SCHED, RH>;
  constexpr int RHO = Sh::RHO, R = Sh::R, T = Sh::T, G = Sh::G, G1 = Sh::G1;
  if constexpr (PREC == PREC_FP32) {
#pragma unroll
    for (int i = 0; i < (1 << G1) - 1; ++i) ts.w1[i] = make_uniform(tw[i]);
  }
  if constexpr (Sh::TW_REGS) {
#pragma unroll
    for (int g = 2; g <= G; ++g) {
      const int lo = Sh::lo(g);
      const int a_hi = tau >> lo;
#pragma unroll
      for (int t = 0; t < RHO; ++t) {
        // (a loop from 0 unrolls completely, keeping ts.wg in registers)
        if (t < Sh::t0(g)) continue;
        const int u = S - lo - RHO + 1 + t;
#pragma unroll
        for (int h = 0; h < (1 << t); ++h)
          ts.wg[(g - 2) * (R - 1) + (1 << t) - 1 + h] =
              tw[((1 << (u - 1)) - 1) + (a_hi << t) + h];
      }
    }
  }
#pragma unroll
  for (int c = 0; c < R; c += 2) {
    const uint32_t lo16 = src[c * T + tau];
    const uint32_t hi16 = c + 1 < R ? src[(c + 1) * T + tau] : 0u;
    ts.srcpk[c >> 1] = lo16 | (hi16 << 16);
  }
}

template <int S, int SCHED, int RH, int PREC, bool PARTIAL = false>
__global__ void __launch_bounds__((FusedShape<S, SCHED, RH>::THREADS))
hidft_fused_kernel(const float2* __restrict__ in, int64_t ld_in, float2* __restrict__ out,
                   int64_t ld_out, uint64_t batch, const float2* __restrict__ tw,
                   const uint16_t* __restrict__ src, const uint4* __restrict__ amat,
                   float scale, uint32_t n_out) {
  using Sh = FusedShape<S, SCHED, RH>;
  constexpr int R = Sh::R, T = Sh::T, SPB = Sh::SPB;
  extern __shared__ float2 lds[];

  const int tid = threadIdx.x;
  const int slot = tid / T;
  const int tau = tid - slot * T;
  const uint64_t n_groups = (batch + SPB - 1) / SPB;
  MfmaOps<PREC, mfma_blocks<RH>()> op;
  if constexpr (PREC != PREC_FP32) op = load_mfma_ops<PREC, mfma_blocks<RH>()>(amat);

  if constexpr (Sh::BIG) {
    // One signal per block, one block per signal (see BIG above).
    static_assert(SPB == 1, "a large signal fills its block");
    const uint64_t grp = blockIdx.x;
    float2 v[R];
    __builtin_amdgcn_s_setprio(2);
    load_group1<S, SCHED, RH, PREC>(v, in, ld_in, grp, batch);
    __builtin_amdgcn_s_setprio(0);
    const FlatMemT<PARTIAL> mem{tw, src, out + grp * (uint64_t)ld_out, n_out};
    ThreadState<S, SCHED, RH> unused;
    transform_signal<S, SCHED, RH, PREC, false>(v, lds, 0, tau, true, mem, scale, unused, op);
  } else {
    ThreadState<S, SCHED, RH> ts;
    load_thread_state<S, SCHED, RH, PREC>(ts, tw, src, tau);
    float2 vn[R];
    uint64_t grp = blockIdx.x;
    if (grp < n_groups) load_group1<S, SCHED, RH, PREC>(vn, in, ld_in, grp * SPB, batch);
    for (; grp < n_groups; grp += gridDim.x) {
      float2 v[R];
#pragma unroll
      for (int c = 0; c < R; ++c) v[c] = vn[c];
      // Wave priority 2 while the loads are issued (note on wave priority above).
      __builtin_amdgcn_s_setprio(2);
      if (grp + gridDim.x < n_groups)
        load_group1<S, SCHED, RH, PREC>(vn, in, ld_in, (grp + gridDim.x) * SPB, batch);
      __builtin_amdgcn_s_setprio(0);
      const uint64_t sig = grp * SPB + slot;
      const FlatMemT<PARTIAL> mem{tw, src, out + (sig < batch ? sig : 0) * (uint64_t)ld_out,
                                  n_out};
      transform_signal<S, SCHED, RH, PREC, true>(v, lds, slot, tau, sig < batch, mem, scale,
                                                  ts, op);
      lds_barrier();  // the next group overwrites these LDS slots
    }
  }
}

// k = 1: the single coefficient is N f(0) (Algorithm 1, base case, times N/k).
__global__ void hidft_k1_kernel(const float2* __restrict__ in, int64_t ld_in,
                                float2* __restrict__ out, int64_t ld_out, uint64_t batch,
                                float scale) {
  const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const float2 x = in[b * (uint64_t)ld_in];
  out[b * (uint64_t)ld_out] = make_float2(x.x * scale, x.y * scale);
}

// ---------------------------------------------------------------------------
// Inverse transform: coefficients on J (caller's order) -> samples on I_r
// (ascending), f_I = F^{-1}(I_r, J) c = (1/N) F(J, I_r)^H c.
//
// F(J, I_r) in the kernels' orders is the product of the S butterfly stages,
// so its adjoint runs the stages in reverse with each butterfly transposed
// and conjugated: (X, Y) -> (X + Y, conj(w) (X - Y)).  The coefficients are
// scattered through the same gather table (its inverse permutation), the
// radix-16 groups run from the lowest bits up, and the last group (the top
// bits, group 1 of the forward kernel) stores straight to the output rows in
// ascending sample order, scaled by 1/N.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void butterfly_adj(float2& X, float2& Y, const float2 w) {
  const float dr = X.x - Y.x, di = X.y - Y.y;
  X.x += Y.x;
  X.y += Y.y;
  Y.x = fmaf(w.x, dr, w.y * di);
  Y.y = fmaf(w.x, di, -w.y * dr);
}

// Adjoint of transform_signal for one signal: v holds this thread's
// coefficients t = c*T + tau (the caller's order of J).  They are scattered to
// their positions src[t] (the inverse of the forward gather), the groups run
// from the last to the first, each stage reversed within its group, and group
// 1 leaves the samples in registers (positions a = tau + c*T, ascending I_r).
template <int S, int SCHED, bool HOISTED, class Mem>
__device__ __forceinline__ void inverse_signal(SigVec<S, 4>& v, float2* L, int tau,
                                               const Mem& mem,
                                               const ThreadState<S, SCHED, 4>& ts) {
  using Sh = FusedShape<S, SCHED, 4>;
  constexpr int RHO = Sh::RHO, R = Sh::R, T = Sh::T, G = Sh::G, G1 = Sh::G1;
#pragma unroll
  for (int c = 0; c < R; ++c) {
    const int p = HOISTED ? (int)((ts.srcpk[c >> 1] >> (16 * (c & 1))) & 0xffffu)
                          : mem.src_at(c * T, tau);
    L[lds_pad<RHO>(p)] = v[c];
  }
#pragma unroll
  for (int g = G; g >= 2; --g) {
    const int lo = Sh::lo(g), t0 = Sh::t0(g);
    const int a_lo = tau & ((1 << lo) - 1);
    const int a_hi = tau >> lo;
    const int base = a_lo + (a_hi << (lo + RHO));
    float2 wq[R > 1 ? R - 1 : 1];
    if constexpr (!(HOISTED && Sh::TW_REGS)) {
      if constexpr (FirstTwOf<Mem>::value) {
        if (g == G) {
#pragma unroll
          for (int i = 0; i < (R > 1 ? R - 1 : 1); ++i) wq[i] = mem.first_tw[i];
        } else {
          adjoint_group_twiddles<S, SCHED>(wq, mem, tau, g);
        }
      } else {
        adjoint_group_twiddles<S, SCHED>(wq, mem, tau, g);
      }
    }
    lds_barrier();
    const int pb = lds_pad<RHO>(base);
#pragma unroll
    for (int c = 0; c < R; ++c) v[c] = L[pb + lds_window_off<RHO>(c, lo)];
#pragma unroll
    for (int t = RHO - 1; t >= 0; --t) {
      if (t < t0) continue;
      const int bit = RHO - 1 - t;
#pragma unroll
      for (int c = 0; c < R; ++c) {
        if (c & (1 << bit)) continue;
        const int h = c >> (RHO - t);
        float2 w;
        if constexpr (HOISTED && Sh::TW_REGS)
          w = ts.wg[(g - 2) * (R - 1) + (1 << t) - 1 + h];
        else
          w = wq[(1 << t) - 1 + h];
        butterfly_adj(v[c], v[c | (1 << bit)], w);
      }
    }
#pragma unroll
    for (int c = 0; c < R; ++c) L[pb + lds_window_off<RHO>(c, lo)] = v[c];
  }
  lds_barrier();
  if constexpr (T % R == 0) {
    const int pt = lds_pad<RHO>(tau);
#pragma unroll
    for (int c = 0; c < R; ++c) v[c] = L[pt + lds_column_off<RHO>(c, T)];
  } else {
#pragma unroll
    for (int c = 0; c < R; ++c) v[c] = L[lds_pad<RHO>(c * T + tau)];
  }
#pragma unroll
  for (int u = G1; u >= 1; --u) {
    const int bit = RHO - u;
#pragma unroll
    for (int c = 0; c < R; ++c) {
      if (c & (1 << bit)) continue;
      const int idx = (1 << (u - 1)) - 1 + (c >> (bit + 1));
      butterfly_adj(v[c], v[c | (1 << bit)], HOISTED ? ts.w1[idx] : mem.tw_at(idx, 0));
    }
  }
}

// Inverse transform with the forward kernel's shapes: persistent with the
// next signal prefetched and the tables in registers up to 2^13 points, one
// signal per block at 2^14.
template <int S, int SCHED>
__global__ void __launch_bounds__((FusedShape<S, SCHED, 4>::THREADS))
hidft_inverse_kernel(const float2* __restrict__ in, int64_t ld_in, float2* __restrict__ out,
                     int64_t ld_out, uint64_t batch, const float2* __restrict__ tw,
                     const uint16_t* __restrict__ src, float scale) {
  using Sh = FusedShape<S, SCHED, 4>;
  constexpr int R = Sh::R, T = Sh::T, SPB = Sh::SPB;
  extern __shared__ float2 lds[];
  const int tid = threadIdx.x;
  const int slot = tid / T;
  const int tau = tid - slot * T;
  float2* L = lds + slot * Sh::PADK;
  // Wave priorities as in the forward kernel: 2 while issuing loads, 1 for
  // the stores, 0 for the transform.
  auto store = [&](const float2 (&v)[R], uint64_t sig) {
    __builtin_amdgcn_s_setprio(1);
    if (sig < batch) {
      float2* orow = out + sig * (uint64_t)ld_out;
#pragma unroll
      for (int c = 0; c < R; ++c)
        store_stream(orow + c * T + tau, make_float2(v[c].x * scale, v[c].y * scale));
    }
    __builtin_amdgcn_s_setprio(0);
  };
  if constexpr (Sh::BIG) {
    const uint64_t sig = blockIdx.x;
    AdjointMem<R, T> mem;
    mem.tw = tw;
    mem.read_places(src, tau);  // ahead of the signal
    mem.template read_first_twiddles<S, SCHED>(tau);
    float2 v[R];
    __builtin_amdgcn_s_setprio(2);
    load_group1<S, SCHED, 4, PREC_FP32>(v, in, ld_in, sig, batch);
    __builtin_amdgcn_s_setprio(0);
    ThreadState<S, SCHED, 4> unused;
    inverse_signal<S, SCHED, false>(v, L, tau, mem, unused);
    store(v, sig);
  } else {
    const uint64_t n_groups = (batch + SPB - 1) / SPB;
    ThreadState<S, SCHED, 4> ts;
    load_thread_state<S, SCHED, 4, PREC_FP32>(ts, tw, src, tau);
    const FlatMem mem{tw, src, nullptr, 0};
    float2 vn[R];
    uint64_t grp = blockIdx.x;
    if (grp < n_groups) load_group1<S, SCHED, 4, PREC_FP32>(vn, in, ld_in, grp * SPB, batch);
    for (; grp < n_groups; grp += gridDim.x) {
      float2 v[R];
#pragma unroll
      for (int c = 0; c < R; ++c) v[c] = vn[c];
      __builtin_amdgcn_s_setprio(2);
      if (grp + gridDim.x < n_groups)
        load_group1<S, SCHED, 4, PREC_FP32>(vn, in, ld_in, (grp + gridDim.x) * SPB, batch);
      __builtin_amdgcn_s_setprio(0);
      inverse_signal<S, SCHED, true>(v, L, tau, mem, ts);
      store(v, grp * SPB + slot);
      lds_barrier();  // the next group of signals overwrites these LDS slots
    }
  }
}

template <int S>
static hipError_t launch_inverse_s(const float2* in, int64_t ld_in, float2* out, int64_t ld_out,
                                   uint64_t batch, const float2* tw, const uint16_t* src,
                                   float scale, hipStream_t stream) {
  // The adjoint of hidft_execute's default grouping (short group last).
  constexpr int SC = S > 4 && S % 4 != 0 ? SCHED_SHORT_LAST : SCHED_SHORT_FIRST;
  using Sh = FusedShape<S, SC, 4>;
  static OccupancyCache cache;
  Occupancy occ;
  if (!cache.get(&occ)) {
    hipError_t e = query_occupancy((const void*)hidft_inverse_kernel<S, SC>, Sh::THREADS,
                                   Sh::LDS_BYTES, &occ);
    if (e != hipSuccess) return e;
    cache.put(occ);
  }
  if constexpr (Sh::BIG) {
    const uint64_t chunk = 0x7fffffffULL;  // one block per signal
    for (uint64_t first = 0; first < batch; first += chunk) {
      const uint64_t n = batch - first < chunk ? batch - first : chunk;
      hipLaunchKernelGGL((hidft_inverse_kernel<S, SC>), dim3((unsigned)n), dim3(Sh::THREADS),
                         Sh::LDS_BYTES, stream, in + first * (uint64_t)ld_in, ld_in,
                         out + first * (uint64_t)ld_out, ld_out, n, tw, src, scale);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const uint64_t max_grid = (uint64_t)occ.per_cu * (uint64_t)occ.cus;
  const uint64_t groups = (batch + Sh::SPB - 1) / Sh::SPB;
  const unsigned grid = (unsigned)(groups < max_grid ? groups : max_grid);
  hipLaunchKernelGGL((hidft_inverse_kernel<S, SC>), dim3(grid), dim3(Sh::THREADS), Sh::LDS_BYTES,
                     stream, in, ld_in, out, ld_out, batch, tw, src, scale);
  return hipGetLastError();
}

hipError_t launch_inverse(uint32_t s, const float2* in, int64_t ld_in, float2* out,
                          int64_t ld_out, uint64_t batch, const float2* tw, const uint16_t* src,
                          float scale, hipStream_t stream) {
  if (batch == 0) return hipSuccess;
  switch (s) {
    case 0: {
      const uint64_t blocks = (batch + 255) / 256;
      if (blocks > 0x7fffffffULL) return hipErrorInvalidValue;
      hipLaunchKernelGGL(hidft_k1_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, in,
                         ld_in, out, ld_out, batch, scale);
      return hipGetLastError();
    }
#define HIDFT_CASE(S) \
  case S:             \
    return launch_inverse_s<S>(in, ld_in, out, ld_out, batch, tw, src, scale, stream);
    HIDFT_CASE(1) HIDFT_CASE(2) HIDFT_CASE(3) HIDFT_CASE(4) HIDFT_CASE(5) HIDFT_CASE(6)
    HIDFT_CASE(7) HIDFT_CASE(8) HIDFT_CASE(9) HIDFT_CASE(10) HIDFT_CASE(11) HIDFT_CASE(12)
    HIDFT_CASE(13) HIDFT_CASE(14)
#undef HIDFT_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <int S, int SCHED, int RH, int PREC, bool PARTIAL = false>
static hipError_t launch_fused_s(const float2* in, int64_t ld_in, float2* out, int64_t ld_out,
                                 uint64_t batch, const float2* tw, const uint16_t* src,
                                 const uint4* amat, float scale, uint32_t n_out,
                                 int blocks_per_cu, hipStream_t stream) {
  using Sh = FusedShape<S, SCHED, RH>;
  const void* kernel = (const void*)hidft_fused_kernel<S, SCHED, RH, PREC, PARTIAL>;
  static OccupancyCache cache;
  Occupancy occ;
  if (!cache.get(&occ)) {
    hipError_t e = query_occupancy(kernel, Sh::THREADS, Sh::LDS_BYTES, &occ);
    if (e != hipSuccess) return e;
    cache.put(occ);
  }
  if constexpr (Sh::BIG) {
    // One block per signal: launch in chunks that fit the grid dimension.
    const uint64_t chunk = 0x7fffffffULL;
    for (uint64_t first = 0; first < batch; first += chunk) {
      const uint64_t n = batch - first < chunk ? batch - first : chunk;
      hipLaunchKernelGGL((hidft_fused_kernel<S, SCHED, RH, PREC, PARTIAL>), dim3((unsigned)n),
                         dim3(Sh::THREADS), Sh::LDS_BYTES, stream, in + first * (uint64_t)ld_in,
                         ld_in, out + first * (uint64_t)ld_out, ld_out, n, tw, src, amat, scale,
                         n_out);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const int per_cu =
      blocks_per_cu > 0 && blocks_per_cu < occ.per_cu ? blocks_per_cu : occ.per_cu;
  const uint64_t max_grid = (uint64_t)per_cu * (uint64_t)occ.cus;
  const uint64_t groups = (batch + Sh::SPB - 1) / Sh::SPB;
  const unsigned grid = (unsigned)(groups < max_grid ? groups : max_grid);
  hipLaunchKernelGGL((hidft_fused_kernel<S, SCHED, RH, PREC, PARTIAL>), dim3(grid),
                     dim3(Sh::THREADS),
                     Sh::LDS_BYTES, stream, in, ld_in, out, ld_out, batch, tw, src, amat, scale,
                     n_out);
  return hipGetLastError();
}

bool fused_variant_exists(uint32_t s, int sched, int prec, int rho) {
  if (s > HIDFT_MAX_LOG2_K_DEVICE) return false;
  if (sched != SCHED_SHORT_FIRST && sched != SCHED_SHORT_LAST) return false;
  if (rho != 4 && rho != 5) return false;
  if (prec != PREC_FP32 && prec != PREC_F16X2 && prec != PREC_BF16X3) return false;
  // Radix-32 tiles exist for the one-signal-per-block sizes; the matrix-core
  // group 1 is then a full radix-32 group (short group last).
  if (rho == 5) return s >= 13 && (prec == PREC_FP32 || sched == SCHED_SHORT_LAST);
  if (prec == PREC_FP32) return true;
  // Matrix-core group 1 is a full radix-16 group.
  return s >= 4 && (sched == SCHED_SHORT_LAST || s % 4 == 0);
}

template <int S>
static hipError_t dispatch_fused(const float2* in, int64_t ld_in, float2* out, int64_t ld_out,
                                 uint64_t batch, const float2* tw, const uint16_t* src,
                                 const uint4* amat, float scale, uint32_t n_out,
                                 const ExecConfig& cfg, hipStream_t stream) {
  const int bpc = cfg.blocks_per_cu;
  const bool last = cfg.sched == SCHED_SHORT_LAST;
  // When 4 divides S (or S < 4) the two schedules are the same kernel.
  constexpr bool TWO_SCHEDS = S > 4 && S % 4 != 0;
  if (n_out < (1u << S)) {
    // Partial output exists for the default variant (FP32, short group last).
    if (cfg.prec != PREC_FP32 || cfg.rho != 4 || !last) return hipErrorInvalidValue;
    constexpr int SC = TWO_SCHEDS ? SCHED_SHORT_LAST : SCHED_SHORT_FIRST;
    return launch_fused_s<S, SC, 4, PREC_FP32, true>(in, ld_in, out, ld_out, batch, tw, src,
                                                     amat, scale, n_out, bpc, stream);
  }
  if constexpr (S >= 13) {
    if (cfg.rho == 5) {
      // Radix 32: 13 = 3 + 5 + 5 or 5 + 5 + 3, 14 = 4 + 5 + 5 or 5 + 5 + 4.
      if (cfg.prec == PREC_F16X2)
        return launch_fused_s<S, SCHED_SHORT_LAST, 5, PREC_F16X2>(in, ld_in, out, ld_out, batch,
                                                                  tw, src, amat, scale, n_out,
                                                                  bpc, stream);
      if (cfg.prec == PREC_BF16X3)
        return launch_fused_s<S, SCHED_SHORT_LAST, 5, PREC_BF16X3>(in, ld_in, out, ld_out,
                                                                   batch, tw, src, amat, scale,
                                                                   n_out, bpc, stream);
      if (last)
        return launch_fused_s<S, SCHED_SHORT_LAST, 5, PREC_FP32>(in, ld_in, out, ld_out, batch,
                                                                 tw, src, amat, scale, n_out, bpc,
                                                                 stream);
      return launch_fused_s<S, SCHED_SHORT_FIRST, 5, PREC_FP32>(in, ld_in, out, ld_out, batch,
                                                                tw, src, amat, scale, n_out, bpc, stream);
    }
  }
  if (cfg.prec == PREC_FP32) {
    if constexpr (TWO_SCHEDS) {
      if (last)
        return launch_fused_s<S, SCHED_SHORT_LAST, 4, PREC_FP32>(in, ld_in, out, ld_out, batch,
                                                                 tw, src, amat, scale, n_out, bpc,
                                                                 stream);
    }
    return launch_fused_s<S, SCHED_SHORT_FIRST, 4, PREC_FP32>(in, ld_in, out, ld_out, batch, tw,
                                                              src, amat, scale, n_out, bpc, stream);
  }
  if constexpr (S >= 4) {
    constexpr int SC = TWO_SCHEDS ? SCHED_SHORT_LAST : SCHED_SHORT_FIRST;
    if (cfg.prec == PREC_F16X2)
      return launch_fused_s<S, SC, 4, PREC_F16X2>(in, ld_in, out, ld_out, batch, tw, src, amat,
                                                  scale, n_out, bpc, stream);
    if (cfg.prec == PREC_BF16X3)
      return launch_fused_s<S, SC, 4, PREC_BF16X3>(in, ld_in, out, ld_out, batch, tw, src, amat,
                                                   scale, n_out, bpc, stream);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_fused(uint32_t s, const float2* in, int64_t ld_in, float2* out,
                        int64_t ld_out, uint64_t batch, const float2* tw, const uint16_t* src,
                        const void* amat, float scale, ExecConfig cfg, hipStream_t stream,
                        uint32_t n_out) {
  if (!fused_variant_exists(s, cfg.sched, cfg.prec, cfg.rho)) return hipErrorInvalidValue;
  if (cfg.prec != PREC_FP32 && amat == nullptr) return hipErrorInvalidValue;
  if (batch == 0) return hipSuccess;
  const uint32_t k = 1u << s;
  if (n_out == 0 || n_out > k) n_out = k;
  const uint4* am = static_cast<const uint4*>(amat);
  switch (s) {
    case 0: {
      const uint64_t blocks = (batch + 255) / 256;
      if (blocks > 0x7fffffffULL) return hipErrorInvalidValue;
      hipLaunchKernelGGL(hidft_k1_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, in,
                         ld_in, out, ld_out, batch, scale);
      return hipGetLastError();
    }
#define HIDFT_CASE(S) \
  case S:             \
    return dispatch_fused<S>(in, ld_in, out, ld_out, batch, tw, src, am, scale, n_out, cfg, \
                             stream);
    HIDFT_CASE(1) HIDFT_CASE(2) HIDFT_CASE(3) HIDFT_CASE(4) HIDFT_CASE(5) HIDFT_CASE(6)
    HIDFT_CASE(7) HIDFT_CASE(8) HIDFT_CASE(9) HIDFT_CASE(10) HIDFT_CASE(11) HIDFT_CASE(12)
    HIDFT_CASE(13) HIDFT_CASE(14)
#undef HIDFT_CASE
    default:
      return hipErrorInvalidValue;
  }
}

size_t fused_lds_bytes(uint32_t s) {
  switch (s) {
#define HIDFT_CASE(S) \
  case S:             \
    return FusedShape<S>::LDS_BYTES;
    HIDFT_CASE(1) HIDFT_CASE(2) HIDFT_CASE(3) HIDFT_CASE(4) HIDFT_CASE(5) HIDFT_CASE(6)
    HIDFT_CASE(7) HIDFT_CASE(8) HIDFT_CASE(9) HIDFT_CASE(10) HIDFT_CASE(11) HIDFT_CASE(12)
    HIDFT_CASE(13) HIDFT_CASE(14)
#undef HIDFT_CASE
    default:
      return 0;
  }
}

// ---------------------------------------------------------------------------
// Grouped transform: an uneven batch (each instance with its own plan and
// size) in one persistent launch.
//
// Wide phase.  Instances of 2^13 and 2^14 points go in packs that fill the
// whole block (1024 threads, up to 2^14 points and 136 KB of LDS: one block
// per CU); the blocks walk the wide packs with a grid stride.
// Narrow phase.  Then each block splits into four 256-thread sub-blocks
// (lanes) with a quarter of the LDS each and their own barriers (an LDS
// counter), and each lane runs the narrow packs (instances of up to 2^12
// points, packed into at most 2^12 points) that the host's schedule gave it.
// The lanes progress independently, so the load, transform and store phases
// of four packs overlap on a CU, as four fused blocks would.  (A device-wide
// work queue instead cost more in same-address atomics than it gained in
// balance: 74 us against 38.5 us on the uneven configuration.)
// Every instance runs the fused kernel's per-signal code (transform_signal),
// so its result is bit-identical to hidft_execute's.
// ---------------------------------------------------------------------------
constexpr int GROUPED_THREADS = 1024;
constexpr int GROUPED_LDS_SLOTS = (1 << HIDFT_MAX_LOG2_K_DEVICE) + ((1 << HIDFT_MAX_LOG2_K_DEVICE) >> 4);
constexpr int NARROW_THREADS = 256;
constexpr int NARROW_SUBBLOCKS = GROUPED_THREADS / NARROW_THREADS;
static_assert(NARROW_SUBBLOCKS == (int)GROUP_NARROW_PER_BLOCK, "sub-blocks per block");
constexpr int NARROW_LDS_SLOTS = GROUPED_LDS_SLOTS / NARROW_SUBBLOCKS;  // 2^12 + 2^8
static_assert(NARROW_LDS_SLOTS >= (1 << 12) + (1 << 8), "a narrow pack's LDS");
// After the transform areas: the sub-blocks' barrier counters (one word
// each), then the descriptor of a one-instance launch, in float2 slots.
constexpr int GROUPED_CTL_SLOTS = NARROW_SUBBLOCKS / 2;
constexpr int GROUPED_ONE_SLOTS = (int)((sizeof(GroupSlot) + sizeof(float2) - 1) / sizeof(float2));
static_assert(alignof(GroupSlot) <= sizeof(float2), "descriptor alignment in LDS");
constexpr size_t GROUPED_LDS_BYTES =
    (size_t)(GROUPED_LDS_SLOTS + GROUPED_CTL_SLOTS + GROUPED_ONE_SLOTS) * sizeof(float2);

// Pointers into LDS, typed so: the compiler then emits LDS instructions
// through them also in a function that is not inlined into the kernel (a
// plain pointer there would give flat accesses, each of which waits for the
// wavefront's outstanding global loads too).
template <typename T>
using lds_ptr = __attribute__((address_space(3))) T*;

template <typename T>
__device__ __forceinline__ lds_ptr<T> to_lds(T* p) {
  return (lds_ptr<T>)p;
}

// The same for global memory: the descriptors the grouped kernel reads
// hold plain pointers, through which the compiler would emit flat accesses
// (which also count against the LDS wait counter).
template <typename T>
using glb_ptr = __attribute__((address_space(1))) T*;

template <typename T>
__device__ __forceinline__ glb_ptr<T> to_glb(T* p) {
  return (glb_ptr<T>)p;
}

// Per-lane table and output accesses of an instance with fewer than 64
// threads (its rows are not wave-uniform), through global pointers.
struct GlbMem {
  glb_ptr<const f2v_t> tw;
  glb_ptr<const uint16_t> src;
  glb_ptr<f2v_t> out;
  __device__ __forceinline__ float2 tw_at(int uni, int lane) const {
    return __builtin_bit_cast(float2, tw[uni + lane]);
  }
  __device__ __forceinline__ int src_at(int uni, int lane) const { return src[uni + lane]; }
  __device__ __forceinline__ void put(int uni, int lane, float2 x) const {
    __builtin_nontemporal_store(__builtin_bit_cast(f2v_t, x), out + uni + lane);
  }
};

// Barrier of one 256-thread sub-block (four wavefronts) through an LDS
// counter: at each sync every wave adds 1 and waits until the counter reaches
// the next multiple of 4 above the value it found.  That multiple is reached
// exactly when all four waves have arrived, and no wave can arrive at the
// following sync before then, so the target needs no state of its own.
struct SubSync {
  lds_ptr<uint32_t> cnt;
  __device__ __forceinline__ void sync() const {
    constexpr uint32_t W = NARROW_THREADS / 64;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    uint32_t old = 0;
    if ((threadIdx.x & 63) == 0)
      old = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    old = __builtin_amdgcn_readfirstlane(old);
    const uint32_t target = (old & ~(W - 1)) + W;
    while ((int32_t)(__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) -
                     target) < 0)
      __builtin_amdgcn_s_sleep(1);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  }
};

// A descriptor field that is the same in every lane of the wavefront (a slot
// spans whole wavefronts when T >= 64), moved to scalar registers.
template <typename P>
__device__ __forceinline__ P* uniform_ptr(P* p) {
  const uint64_t x = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return reinterpret_cast<P*>(((uint64_t)hi << 32) | lo);
}

// One pack of 2^S-point instances, short group first or last (SC), on
// THREADS threads (the block, or a sub-block) whose thread index is `tid` and
// whose barrier is `sync`.  Not inlined: each size gets a register
// allocation of its own instead of one shared by the whole switch.
//
// skip_idle (GROUP_SKIP_IDLE): a wavefront whose slots are all empty does no
// arithmetic and only takes part in the transform's barriers, one per group
// after the first and one before the gather (G in all, 1 for S <= 4), the
// same count as the other wavefronts.  The condition is uniform over the
// wavefront (scalar branch).  Measured: in the server's batches, mostly
// single requests, p50 latency 25 -> 22 us; in the partial packs of the
// uneven configuration 38.5 -> 39.3 us, so only the server sets it.
template <int S, int SC, int THREADS, class Sync>
__device__ __attribute__((noinline)) void grouped_pack(const GroupSlot* __restrict__ slots,
                                                       int n_slots, lds_ptr<float2> lds_as,
                                                       int skip_idle, int tid, Sync sync) {
  float2* lds = (float2*)lds_as;
  using Sh = FusedShape<S, SC, 4>;
  constexpr int R = Sh::R, T = Sh::T;
  static_assert(T <= THREADS && THREADS % T == 0, "instances tile the threads");
  constexpr uint32_t K = 1u << S;
  const int slot = tid / T;
  const int tau = tid - slot * T;
  const bool valid = slot < n_slots;
  if (__builtin_amdgcn_readfirstlane(skip_idle) &&
      __builtin_amdgcn_readfirstlane((tid & ~63) / T) >=
          __builtin_amdgcn_readfirstlane(n_slots)) {
    constexpr int NB = Sh::G > 1 ? Sh::G : 1;
#pragma unroll
    for (int i = 0; i < NB; ++i) sync.sync();
    return;
  }
  // Threads of empty slots (a partial pack) run the transform on zeros with
  // slot 0's tables (every pack has at least one slot) and store nothing.
  GroupSlot d = slots[valid ? slot : 0];
  float2 v[R];
  ThreadState<S, SC, 4> unused;
  const MfmaOps<PREC_FP32> no_mfma;
  if constexpr (T >= 64) {
    // A slot spans whole wavefronts: its descriptor is wave-uniform.
    d.in = uniform_ptr(d.in);
    d.out = uniform_ptr(d.out);
    d.tw = uniform_ptr(d.tw);
    d.src = uniform_ptr(d.src);
    d.scale = __builtin_bit_cast(
        float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(uint32_t, d.scale)));
    if (valid) {
      load_row<R, T, true>(v, d.in, K);
    } else {
#pragma unroll
      for (int c = 0; c < R; ++c) v[c] = make_float2(0.f, 0.f);
    }
    BufMem mem;
    mem.tw = make_rsrc(d.tw, (K > 1 ? K - 1 : 1) * 8u);
    mem.src = make_rsrc(d.src, K * 2u);
    mem.out = make_rsrc(d.out, K * 8u);
    transform_signal<S, SC, 4, PREC_FP32, false, BufMem, Sync>(v, lds, slot, tau, valid, mem,
                                                               d.scale, unused, no_mfma, sync);
  } else {
    const glb_ptr<const f2v_t> in = to_glb(reinterpret_cast<const f2v_t*>(d.in));
#pragma unroll
    for (int c = 0; c < R; ++c)
      v[c] = valid ? __builtin_bit_cast(float2, __builtin_nontemporal_load(in + c * T + tau))
                   : make_float2(0.f, 0.f);
    const GlbMem mem{to_glb(reinterpret_cast<const f2v_t*>(d.tw)), to_glb(d.src),
                     to_glb(reinterpret_cast<f2v_t*>(d.out))};
    transform_signal<S, SC, 4, PREC_FP32, false, GlbMem, Sync>(v, lds, slot, tau, valid, mem,
                                                               d.scale, unused, no_mfma, sync);
  }
}

// The whole block runs wide pack `code` (a GroupPack::log2_k) of n slots.
__device__ __forceinline__ void run_wide_pack(uint32_t code, const GroupSlot* sl, int n,
                                              lds_ptr<float2> L, int tid) {
  // Sizes with two schedules (S > 4, 4 does not divide S) have a body for
  // each; the others ignore the flag.
  const int skip = (code & GROUP_SKIP_IDLE) != 0;
  switch (code & ~GROUP_SKIP_IDLE) {
    case 13:
      grouped_pack<13, SCHED_SHORT_LAST, GROUPED_THREADS>(sl, n, L, skip, tid, BlockSync());
      break;
    case 13 | GROUP_SHORT_FIRST:
      grouped_pack<13, SCHED_SHORT_FIRST, GROUPED_THREADS>(sl, n, L, skip, tid, BlockSync());
      break;
    case 14:
      grouped_pack<14, SCHED_SHORT_LAST, GROUPED_THREADS>(sl, n, L, skip, tid, BlockSync());
      break;
    case 14 | GROUP_SHORT_FIRST:
      grouped_pack<14, SCHED_SHORT_FIRST, GROUPED_THREADS>(sl, n, L, skip, tid, BlockSync());
      break;
    default:
      break;
  }
}

// A narrow sub-block (thread stid of NARROW_THREADS, barrier `sync`) runs
// narrow pack `code` of n slots.
__device__ __forceinline__ void run_narrow_pack(uint32_t code, const GroupSlot* sl, int n,
                                                lds_ptr<float2> L, int stid, SubSync sync) {
  const int skip = (code & GROUP_SKIP_IDLE) != 0;
  switch (code & ~GROUP_SKIP_IDLE) {
#define HIDFT_ONE(S)                                                                          \
  case S:                                                                                     \
  case S | GROUP_SHORT_FIRST:                                                                 \
    grouped_pack<S, SCHED_SHORT_FIRST, NARROW_THREADS>(sl, n, L, skip, stid, sync);          \
    break;
#define HIDFT_TWO(S)                                                                          \
  case S:                                                                                     \
    grouped_pack<S, SCHED_SHORT_LAST, NARROW_THREADS>(sl, n, L, skip, stid, sync);           \
    break;                                                                                    \
  case S | GROUP_SHORT_FIRST:                                                                 \
    grouped_pack<S, SCHED_SHORT_FIRST, NARROW_THREADS>(sl, n, L, skip, stid, sync);          \
    break;
    HIDFT_ONE(0) HIDFT_ONE(1) HIDFT_ONE(2) HIDFT_ONE(3) HIDFT_ONE(4) HIDFT_TWO(5)
    HIDFT_TWO(6) HIDFT_TWO(7) HIDFT_ONE(8) HIDFT_TWO(9) HIDFT_TWO(10) HIDFT_TWO(11)
    HIDFT_ONE(12)
#undef HIDFT_ONE
#undef HIDFT_TWO
    default:
      break;
  }
}

// n_few > 0: a launch of n_few blocks for as many instances, block b taking
// instance b, whose descriptor and pack code come with the arguments, so the
// transform starts without reading the pack, slot and lane tables (three
// dependent reads, over the host link when those tables sit in mapped host
// memory as the server's do).  The descriptor is copied to LDS for the pack
// body, which reads its slots through a pointer.
__global__ void __launch_bounds__(GROUPED_THREADS)
hidft_grouped_kernel(const GroupPack* __restrict__ packs, uint32_t n_wide, uint32_t n_narrow,
                     const GroupSlot* __restrict__ slots, const uint32_t* __restrict__ lane_end,
                     uint32_t* done_count, uint32_t count_base, uint32_t* done_flag,
                     uint32_t seq, GroupFew few, uint32_t n_few) {
  extern __shared__ float2 lds[];
  const lds_ptr<uint32_t> ctl = to_lds(reinterpret_cast<uint32_t*>(lds + GROUPED_LDS_SLOTS));
  if (n_few > 0) {
    const uint32_t b = blockIdx.x;  // < n_few: the launch has n_few blocks
    const uint32_t code = few.code[b];
    GroupSlot* od = reinterpret_cast<GroupSlot*>(lds + GROUPED_LDS_SLOTS + GROUPED_CTL_SLOTS);
    if (threadIdx.x == 0) *od = few.slot[b];
    if (threadIdx.x < NARROW_SUBBLOCKS) ctl[threadIdx.x] = 0u;
    lds_barrier();
    if ((code & 0xffu) >= GROUP_WIDE_MIN_S) {
      run_wide_pack(code, od, 1, to_lds(lds), (int)threadIdx.x);
    } else if (threadIdx.x < NARROW_THREADS) {
      // the first sub-block (whole wavefronts) and its barrier counter
      run_narrow_pack(code, od, 1, to_lds(lds), (int)threadIdx.x, SubSync{ctl});
    }
  } else {
    // Wide phase: whole-block packs, grid stride.
    for (uint32_t p = blockIdx.x; p < n_wide; p += gridDim.x) {
      const GroupPack pk = packs[p];
      run_wide_pack(pk.log2_k, slots + pk.first_slot, (int)pk.n_slots, to_lds(lds),
                    (int)threadIdx.x);
      lds_barrier();  // the next pack overwrites the LDS
    }
    if (n_narrow > 0) {
      // Narrow phase: four lanes, each with its own LDS quarter and barrier
      // counter, and its packs [lane_end[lane - 1], lane_end[lane]).
      const int sub = __builtin_amdgcn_readfirstlane(threadIdx.x / NARROW_THREADS);
      const int stid = threadIdx.x % NARROW_THREADS;
      const uint32_t lane = blockIdx.x * NARROW_SUBBLOCKS + sub;
      const uint32_t begin = lane == 0 ? 0u : lane_end[lane - 1];
      const uint32_t end = lane_end[lane];
      if (threadIdx.x < NARROW_SUBBLOCKS) ctl[threadIdx.x] = 0u;
      lds_barrier();
      const SubSync sync{ctl + sub};
      const lds_ptr<float2> L = to_lds(lds + sub * NARROW_LDS_SLOTS);
      for (uint32_t q = begin; q < end; ++q) {
        const GroupPack pk = packs[n_wide + q];
        run_narrow_pack(pk.log2_k, slots + pk.first_slot, (int)pk.n_slots, L, stid, sync);
        sync.sync();  // the next pack overwrites this lane's LDS
      }
    }
  }
  if (done_flag != nullptr) {
    // Completion signal (the server's batches): every block makes its stores
    // visible at system scope, then counts itself on done_count, which only
    // grows (count_base = its value before this launch); the last block
    // stores seq to the host-mapped flag.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    __syncthreads();
    if (threadIdx.x == 0) {
      const uint32_t old = __hip_atomic_fetch_add(done_count, 1u, __ATOMIC_ACQ_REL,
                                                  __HIP_MEMORY_SCOPE_AGENT);
      if (old == count_base + gridDim.x - 1) {
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "");
        __hip_atomic_store(done_flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
      }
    }
  }
}

int grouped_slots_per_pack(uint32_t s) {
  if (s >= GROUP_WIDE_MIN_S) return GROUPED_THREADS >> (s - 4);
  return NARROW_THREADS >> (s > 4 ? s - 4 : 0);
}

hipError_t grouped_grid(uint32_t* blocks) {
  // Queried on the first call; racing threads store the same value.
  static std::atomic<int> cached{0};
  int max_grid = cached.load(std::memory_order_acquire);
  if (max_grid == 0) {
    hipError_t e = hipFuncSetAttribute((const void*)hidft_grouped_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)GROUPED_LDS_BYTES);
    if (e != hipSuccess) return e;
    int dev = 0, cus = 0, per_cu = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) !=
        hipSuccess)
      return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
             &per_cu, (const void*)hidft_grouped_kernel, GROUPED_THREADS, GROUPED_LDS_BYTES)) !=
        hipSuccess)
      return e;
    max_grid = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
    cached.store(max_grid, std::memory_order_release);
  }
  *blocks = (uint32_t)max_grid;
  return hipSuccess;
}

hipError_t launch_grouped(const GroupPack* d_packs, uint32_t n_wide, uint32_t n_narrow,
                          const GroupSlot* d_slots, const uint32_t* d_lane_end, uint32_t grid,
                          hipStream_t stream, const GroupDone* done) {
  if (n_wide == 0 && n_narrow == 0) return hipSuccess;
  uint32_t max_grid = 0;
  hipError_t e = grouped_grid(&max_grid);
  if (e != hipSuccess) return e;
  if (grid == 0 || grid > max_grid) return hipErrorInvalidValue;
  hipLaunchKernelGGL(hidft_grouped_kernel, dim3(grid), dim3(GROUPED_THREADS), GROUPED_LDS_BYTES,
                     stream, d_packs, n_wide, n_narrow, d_slots, d_lane_end,
                     done ? done->d_count : nullptr, done ? *done->count_base : 0u,
                     done ? done->d_flag : nullptr, done ? done->seq : 0u, GroupFew{}, 0u);
  e = hipGetLastError();
  if (e == hipSuccess && done) *done->count_base += grid;
  return e;
}

hipError_t launch_grouped_few(const GroupFew& few, uint32_t n, hipStream_t stream,
                              const GroupDone* done) {
  if (n == 0 || n > GROUP_FEW_MAX) return hipErrorInvalidValue;
  for (uint32_t i = 0; i < n; ++i)
    if ((few.code[i] & 0xffu) > HIDFT_MAX_LOG2_K_DEVICE) return hipErrorInvalidValue;
  uint32_t max_grid = 0;
  hipError_t e = grouped_grid(&max_grid);  // sets the kernel's LDS limit
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(hidft_grouped_kernel, dim3(n), dim3(GROUPED_THREADS), GROUPED_LDS_BYTES,
                     stream, nullptr, 0u, 0u, nullptr, nullptr,
                     done ? done->d_count : nullptr, done ? *done->count_base : 0u,
                     done ? done->d_flag : nullptr, done ? done->seq : 0u, few, n);
  e = hipGetLastError();
  if (e == hipSuccess && done) *done->count_base += n;
  return e;
}

// ---------------------------------------------------------------------------
// Shift-and-Sample leaf solves (Algorithm 2, steps 5-7), FP64.
//
// For each node v at level r_max + 1 with elements l_0..l_{mu-1}, the shifted
// Hi-DFTs give y_j(v) = sum_t c_t z_t^j for j < mu* (scaled by N/2^s),
// z_t = e^{2 pi i l_t / N}: the dual Vandermonde system V c = y of
// Eq. alg1_system, V[j][t] = z_t^j, in its first mu(v) rows.  The matrix
// depends on the plan only, so its inverse is formed once, in FP64, at plan
// creation (sas_inverse_kernel: column j is the Bjorck-Pereyra solution for
// the unit vector e_j, O(mu^2) per column), and each signal's solve is one
// row of that inverse times the node's mu values, accumulated in FP64
// (sas_apply_kernel).
// ---------------------------------------------------------------------------
struct cplx64 {
  double x, y;
};
__device__ __forceinline__ cplx64 csub(cplx64 a, cplx64 b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cplx64 cmul(cplx64 a, cplx64 b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ cplx64 cdiv(cplx64 a, cplx64 b) {
  const double d = b.x * b.x + b.y * b.y;
  return {(a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d};
}

// Plan time, one thread per node: inv[off(v) + i*mu + j] = (V_v^{-1})[i][j].
__global__ void __launch_bounds__(64)
sas_inverse_kernel(uint32_t n_nodes, const uint32_t* __restrict__ node_first,
                   const uint32_t* __restrict__ node_count, const uint32_t* __restrict__ inv_off,
                   const uint64_t* __restrict__ elem_val, uint32_t log2_n,
                   cplx64* __restrict__ inv) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_nodes) return;
  const uint32_t mu = node_count[v];
  const uint32_t first = node_first[v];
  cplx64 x[SAS_MAX_MU], z[SAS_MAX_MU];
  for (uint32_t t = 0; t < mu; ++t) {
    // z = exp(2 pi i l / N) = cospi(2l/N) + i sinpi(2l/N); 2l/N = l 2^{1-M} is exact
    // for l < 2^53.
    double sn, cs;
    sincospi(ldexp((double)elem_val[first + t], 1 - (int)log2_n), &sn, &cs);
    z[t] = {cs, sn};
  }
  const int n = (int)mu - 1;
  for (uint32_t col = 0; col < mu; ++col) {
    for (uint32_t t = 0; t < mu; ++t) x[t] = {t == col ? 1.0 : 0.0, 0.0};
    for (int k = 0; k < n; ++k)
      for (int i = n; i > k; --i) x[i] = csub(x[i], cmul(z[k], x[i - 1]));
    for (int k = n - 1; k >= 0; --k) {
      for (int i = k + 1; i <= n; ++i) x[i] = cdiv(x[i], csub(z[i], z[i - k - 1]));
      for (int i = k; i < n; ++i) x[i] = csub(x[i], x[i + 1]);
    }
    for (uint32_t i = 0; i < mu; ++i) inv[inv_off[v] + i * mu + col] = x[i];
  }
}

hipError_t launch_sas_inverse(uint32_t n_nodes, const uint32_t* node_first,
                              const uint32_t* node_count, const uint32_t* inv_off,
                              const uint64_t* elem_val, uint32_t log2_n, void* inv,
                              hipStream_t stream) {
  if (n_nodes == 0) return hipSuccess;
  hipLaunchKernelGGL(sas_inverse_kernel, dim3((n_nodes + 63) / 64), dim3(64), 0, stream,
                     n_nodes, node_first, node_count, inv_off, elem_val, log2_n,
                     static_cast<cplx64*>(inv));
  return hipGetLastError();
}

// Per signal, one thread per element e (elements in node order): the element
// is row i = e - first(v) of node v = elem_node[e]; y is [signal][shift][node].
constexpr int SAS_APPLY_THREADS = 256;

__global__ void __launch_bounds__(SAS_APPLY_THREADS)
sas_apply_kernel(const float2* __restrict__ y, uint32_t n_nodes, uint32_t mu_star,
                 uint64_t batch, uint32_t k, const uint32_t* __restrict__ elem_node,
                 const uint32_t* __restrict__ node_first, const uint32_t* __restrict__ node_count,
                 const uint32_t* __restrict__ inv_off, const cplx64* __restrict__ inv,
                 const uint32_t* __restrict__ elem_t, float2* __restrict__ out, int64_t ld_out) {
  const uint32_t e = blockIdx.x * SAS_APPLY_THREADS + threadIdx.x;
  if (e >= k) return;
  const uint32_t v = elem_node[e];
  const uint32_t mu = node_count[v];
  const cplx64* row = inv + inv_off[v] + (e - node_first[v]) * mu;
  const uint32_t dst = elem_t[e];
  for (uint64_t b = blockIdx.y; b < batch; b += gridDim.y) {
    const float2* yv = y + b * mu_star * (uint64_t)n_nodes + v;
    double ar = 0.0, ai = 0.0;
    for (uint32_t j = 0; j < mu; ++j) {
      const float2 q = yv[(uint64_t)j * n_nodes];
      const cplx64 m = row[j];
      ar = fma(m.x, (double)q.x, fma(-m.y, (double)q.y, ar));
      ai = fma(m.x, (double)q.y, fma(m.y, (double)q.x, ai));
    }
    store_stream(out + b * (uint64_t)ld_out + dst, make_float2((float)ar, (float)ai));
  }
}

// The same solves with one block per signal (grid-stride over the batch),
// for plans whose (mu* n_nodes + k) values fit in SAS_LDS_VALUES:
//   * the signal's mu* rows of node values are loaded into LDS with
//     coalesced reads;
//   * thread x serves the elements x + i * SAS_LDS_THREADS (i < EPT).  Each
//     element's record {node | caller position << 16, offset of its inverse
//     row, mu(v)} is read once per block, so a signal needs only the
//     inverse-row reads (L2-resident), all issued together;
//   * each coefficient is written to its caller position in LDS, and the
//     output row leaves with coalesced stores.
// MU: the row loop unrolled for mu* = 2..4 (elements of smaller nodes skip
// the missing terms), 0 for a loop over mu(v).  The barriers order LDS only.
constexpr int SAS_LDS_THREADS = 512;

template <int EPT, int MU>
__global__ void __launch_bounds__(SAS_LDS_THREADS)
sas_apply_lds_kernel(const float2* __restrict__ y, uint32_t n_nodes, uint32_t mu_star,
                     uint64_t batch, uint32_t k, const uint4* __restrict__ rec,
                     const cplx64* __restrict__ inv, float2* __restrict__ out,
                     int64_t ld_out) {
  extern __shared__ float2 sm[];
  const uint32_t ny = mu_star * n_nodes;
  float2* res = sm + ny;
  uint32_t pos[EPT], row[EPT], cnt[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const uint32_t e = threadIdx.x + i * SAS_LDS_THREADS;
    const uint4 r = e < k ? rec[e] : make_uint4(0u, 0u, 0u, 0u);
    pos[i] = r.x;
    row[i] = r.y;
    cnt[i] = r.z;  // 0: no element
  }
  constexpr int UNROLL = 4;
  for (uint64_t b = blockIdx.x; b < batch; b += gridDim.x) {
    const float2* yb = y + b * (uint64_t)ny;
    for (uint32_t i0 = threadIdx.x; i0 < ny; i0 += UNROLL * SAS_LDS_THREADS) {
      float2 a[UNROLL];
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        const uint32_t i = i0 + u * SAS_LDS_THREADS;
        a[u] = i < ny ? load_stream(yb + i) : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        const uint32_t i = i0 + u * SAS_LDS_THREADS;
        if (i < ny) sm[i] = a[u];
      }
    }
    lds_barrier();
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const uint32_t v = pos[i] & 0xffffu;
      const cplx64* m = inv + row[i];
      double ar = 0.0, ai = 0.0;
      if constexpr (MU > 0) {
        // rows read unconditionally (padded table), terms j < mu(v) summed
        cplx64 w[MU];
#pragma unroll
        for (int j = 0; j < MU; ++j) w[j] = m[j];
#pragma unroll
        for (int j = 0; j < MU; ++j) {
          if ((uint32_t)j < cnt[i]) {
            const float2 q = sm[j * n_nodes + v];
            ar = fma(w[j].x, (double)q.x, fma(-w[j].y, (double)q.y, ar));
            ai = fma(w[j].x, (double)q.y, fma(w[j].y, (double)q.x, ai));
          }
        }
      } else {
        for (uint32_t j = 0; j < cnt[i]; ++j) {
          const float2 q = sm[j * n_nodes + v];
          const cplx64 w = m[j];
          ar = fma(w.x, (double)q.x, fma(-w.y, (double)q.y, ar));
          ai = fma(w.x, (double)q.y, fma(w.y, (double)q.x, ai));
        }
      }
      if (cnt[i] != 0) res[pos[i] >> 16] = make_float2((float)ar, (float)ai);
    }
    lds_barrier();
    float2* ob = out + b * (uint64_t)ld_out;
    for (uint32_t t = threadIdx.x; t < k; t += SAS_LDS_THREADS) store_stream(ob + t, res[t]);
    lds_barrier();  // the next signal overwrites the LDS
  }
}

template <int EPT, int MU>
static hipError_t launch_sas_apply_lds(const float2* y, uint32_t n_nodes, uint32_t mu_star,
                                       uint64_t batch, uint32_t k, const uint4* rec,
                                       const cplx64* inv, float2* out, int64_t ld_out,
                                       hipStream_t stream) {
  // The CU count, queried on the first call; racing threads store the same value.
  static std::atomic<int> cached_cus{0};
  int cus = cached_cus.load(std::memory_order_relaxed);
  if (cus == 0) {
    int dev = 0, c = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    cus = c > 0 ? c : 1;
    cached_cus.store(cus, std::memory_order_relaxed);
  }
  const size_t lds = ((size_t)mu_star * n_nodes + k) * sizeof(float2);
  // Blocks that fit per CU: by LDS (160 KB) and by threads (2048).
  uint64_t per_cu = (160u * 1024u) / (lds ? lds : 1);
  if (per_cu > 2048 / SAS_LDS_THREADS) per_cu = 2048 / SAS_LDS_THREADS;
  if (per_cu == 0) per_cu = 1;
  uint64_t grid = per_cu * (uint64_t)cus;
  if (grid > batch) grid = batch;
  hipLaunchKernelGGL((sas_apply_lds_kernel<EPT, MU>), dim3((unsigned)grid),
                     dim3(SAS_LDS_THREADS), lds, stream, y, n_nodes, mu_star, batch, k, rec, inv,
                     out, ld_out);
  return hipGetLastError();
}

template <int EPT>
static hipError_t launch_sas_apply_lds_mu(const float2* y, uint32_t n_nodes, uint32_t mu_star,
                                          uint64_t batch, uint32_t k, const uint4* rec,
                                          const cplx64* inv, float2* out, int64_t ld_out,
                                          hipStream_t stream) {
  switch (mu_star) {
#define HIDFT_MU(MU)                                                                          \
  case MU:                                                                                    \
    return launch_sas_apply_lds<EPT, MU>(y, n_nodes, mu_star, batch, k, rec, inv, out, ld_out, \
                                         stream);
    HIDFT_MU(2) HIDFT_MU(3) HIDFT_MU(4)  // (mu* = 1 plans take the direct path)
#undef HIDFT_MU
    default:
      return launch_sas_apply_lds<EPT, 0>(y, n_nodes, mu_star, batch, k, rec, inv, out, ld_out,
                                          stream);
  }
}

// ---------------------------------------------------------------------------
// Shift-and-Sample in one kernel (Algorithm 2, steps 2-7) for plans with
// mu* = 2..4 whose node values fit in LDS beside the transform area.
//
// Per signal, the block runs the mu* shifted Hi-DFTs SPB at a time (one per
// signal slot of the fused kernel's shape, with its per-thread tables held
// in registers across the whole batch); each gathers its first n_nodes
// outputs (node order, scaled by N/2^s) into an LDS row of node values
// instead of global memory.  The leaf solves then read those values from
// LDS: thread x serves the elements x + i * THREADS, i < SAS_FUSED_EPT,
// whose records {node | caller position << 16, inverse-row offset, mu(v)}
// it loaded once; each coefficient is written to its caller position in an
// LDS row (over the transform area, or after the node values when k does
// not fit there), which leaves with coalesced stores.  The transforms and
// solves are the two-launch path's, operation for operation, so the results
// are bit-identical to it; what goes away is the workspace round trip
// through HBM (mu* n_nodes values written and read back per signal).
// ---------------------------------------------------------------------------
constexpr int SAS_FUSED_EPT = 8;
constexpr size_t SAS_FUSED_MAX_LDS = 80 * 1024;

template <int S>
struct SasFused {
  static constexpr int SC = (S > 4 && S % 4 != 0) ? SCHED_SHORT_LAST : SCHED_SHORT_FIRST;
  using Sh = FusedShape<S, SC, 4>;
  static constexpr uint32_t TRANSFORM_SLOTS = (uint32_t)(Sh::SPB * Sh::PADK);
  static size_t lds_bytes(uint32_t mu_star, uint32_t n_nodes, uint32_t k) {
    const uint64_t extra = k <= TRANSFORM_SLOTS ? 0 : k;
    return ((uint64_t)TRANSFORM_SLOTS + (uint64_t)mu_star * n_nodes + extra) * sizeof(float2);
  }
};

// Output of a shifted Hi-DFT into LDS: the first n_out outputs of the gather
// order (the nodes) go to y[0 .. n_out).
struct LdsOut {
  const float2* tw;
  const uint16_t* src;
  float2* y;
  uint32_t n_out;
  __device__ __forceinline__ float2 tw_at(int uni, int lane) const { return tw[uni + lane]; }
  __device__ __forceinline__ int src_at(int uni, int lane) const { return src[uni + lane]; }
  __device__ __forceinline__ void put(int uni, int lane, float2 x) const {
    if ((uint32_t)(uni + lane) < n_out) y[uni + lane] = x;
  }
};

template <int S>
__global__ void __launch_bounds__(SasFused<S>::Sh::THREADS)
sas_fused_kernel(const float2* __restrict__ in, int64_t ld_in, float2* __restrict__ out,
                 int64_t ld_out, uint64_t batch, uint32_t mu_star, uint32_t n_nodes, uint32_t k,
                 const float2* __restrict__ tw, const uint16_t* __restrict__ src_node,
                 float scale, const uint4* __restrict__ rec, const cplx64* __restrict__ inv) {
  constexpr int SC = SasFused<S>::SC;
  using Sh = typename SasFused<S>::Sh;
  constexpr int R = Sh::R, T = Sh::T, SPB = Sh::SPB, THREADS = Sh::THREADS;
  constexpr uint32_t K = 1u << S;
  static_assert(!Sh::BIG && Sh::TW_REGS, "the persistent shape holds its tables in registers");
  extern __shared__ float2 lds[];
  float2* yv = lds + SasFused<S>::TRANSFORM_SLOTS;
  float2* res = k <= SasFused<S>::TRANSFORM_SLOTS ? lds : yv + mu_star * n_nodes;
  const int tid = threadIdx.x;
  const int slot = tid / T;
  const int tau = tid - slot * T;
  ThreadState<S, SC, 4> ts;
  load_thread_state<S, SC, 4, PREC_FP32>(ts, tw, src_node, tau);
  uint32_t pos[SAS_FUSED_EPT], row[SAS_FUSED_EPT], cnt[SAS_FUSED_EPT];
#pragma unroll
  for (int i = 0; i < SAS_FUSED_EPT; ++i) {
    const uint32_t e = tid + i * THREADS;
    const uint4 r = e < k ? rec[e] : make_uint4(0u, 0u, 0u, 0u);
    pos[i] = r.x;
    row[i] = r.y;
    cnt[i] = r.z;  // 0: no element
  }
  const MfmaOps<PREC_FP32> no_mfma;
  for (uint64_t b = blockIdx.x; b < batch; b += gridDim.x) {
    const float2* sig = in + b * (uint64_t)ld_in;
    for (uint32_t j0 = 0; j0 < mu_star; j0 += SPB) {
      const uint32_t j = j0 + slot;
      const bool live = j < mu_star;
      float2 v[R];
      if (live) {
        const float2* x = sig + (uint64_t)j * K;
#pragma unroll
        for (int c = 0; c < R; ++c) v[c] = load_stream(x + c * T + tau);
      } else {
#pragma unroll
        for (int c = 0; c < R; ++c) v[c] = make_float2(0.f, 0.f);
      }
      const LdsOut mem{tw, src_node, yv + (live ? j : 0) * n_nodes, n_nodes};
      transform_signal<S, SC, 4, PREC_FP32, true>(v, lds, slot, tau, live, mem, scale, ts,
                                                   no_mfma);
      lds_barrier();  // node values complete; the transform area is free
    }
#pragma unroll
    for (int i = 0; i < SAS_FUSED_EPT; ++i) {
      const uint32_t v = pos[i] & 0xffffu;
      const cplx64* m = inv + row[i];
      double ar = 0.0, ai = 0.0;
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        if ((uint32_t)jj < cnt[i]) {
          const float2 q = yv[jj * n_nodes + v];
          const cplx64 w = m[jj];
          ar = fma(w.x, (double)q.x, fma(-w.y, (double)q.y, ar));
          ai = fma(w.x, (double)q.y, fma(w.y, (double)q.x, ai));
        }
      }
      if (cnt[i] != 0) res[pos[i] >> 16] = make_float2((float)ar, (float)ai);
    }
    lds_barrier();
    float2* ob = out + b * (uint64_t)ld_out;
    for (uint32_t t = tid; t < k; t += THREADS) store_stream(ob + t, res[t]);
    lds_barrier();  // the next signal overwrites the LDS
  }
}

// The one-pass form, for 2^10 and 2^11 points, where the block's signal
// slots hold all mu* shifted transforms of a signal at once (mu* <= SPB).
// The form above keeps each thread's twiddles, gather positions and element
// records in registers for the whole batch and a separate LDS row for the
// node values: 172-180 registers and up to 59 KB of LDS per block, two
// blocks per CU.  Here the tables are read per signal (they stay in the
// caches), each slot's node values are held in registers across the last
// barrier and then written over the transform area, and the coefficients go
// to LDS right after the node values: 145-151 registers and
// max(SPB * PADK, mu* n_nodes + k) slots of LDS, three blocks per CU.  The
// arithmetic is the form above's, operation for operation, so the results
// are the same bits.
template <int T>
struct RegOut {
  const float2* tw;
  const uint16_t* src;
  float2* vals;  // the thread's R outputs, output c * T + tau in vals[c]
  __device__ __forceinline__ float2 tw_at(int uni, int lane) const { return tw[uni + lane]; }
  __device__ __forceinline__ int src_at(int uni, int lane) const { return src[uni + lane]; }
  __device__ __forceinline__ void put(int uni, int, float2 x) const { vals[uni / T] = x; }
};

template <int S>
constexpr bool sas_onepass_shape() { return S == 10 || S == 11; }
// Elements per thread whose reads a solve batch issues together: 8 row
// entries in flight per thread.
template <int MU>
constexpr int sas_solve_batch() { return MU <= 2 ? 4 : 2; }
static_assert(4 <= SAS_INV_PAD, "a row read of mu* <= 4 entries ends in the padding");

template <int S, int MU>
__global__ void __launch_bounds__(SasFused<S>::Sh::THREADS)
sas_onepass_kernel(const float2* __restrict__ in, int64_t ld_in, float2* __restrict__ out,
                   int64_t ld_out, uint64_t batch, uint32_t mu_star, uint32_t n_nodes,
                   uint32_t k, const float2* __restrict__ tw,
                   const uint16_t* __restrict__ src_node, float scale,
                   const uint4* __restrict__ rec, const cplx64* __restrict__ inv) {
  constexpr int SC = SasFused<S>::SC;
  using Sh = typename SasFused<S>::Sh;
  constexpr int R = Sh::R, T = Sh::T, THREADS = Sh::THREADS;
  constexpr uint32_t K = 1u << S;
  extern __shared__ float2 lds[];
  float2* res = lds + mu_star * n_nodes;
  const int tid = threadIdx.x;
  const int slot = tid / T;  // shift j of the signal
  const int tau = tid - slot * T;
  const bool live = (uint32_t)slot < mu_star;
  const MfmaOps<PREC_FP32> no_mfma;
  ThreadState<S, SC, 4> no_state;  // the tables are read per signal
  for (uint64_t b = blockIdx.x; b < batch; b += gridDim.x) {
    float2 v[R];
    if (live) {
      const float2* x = in + b * (uint64_t)ld_in + (uint64_t)slot * K;
#pragma unroll
      for (int c = 0; c < R; ++c) v[c] = load_stream(x + c * T + tau);
    } else {
#pragma unroll
      for (int c = 0; c < R; ++c) v[c] = make_float2(0.f, 0.f);
    }
    float2 vals[R];
    const RegOut<T> mem{tw, src_node, vals};
    transform_signal<S, SC, 4, PREC_FP32, false>(v, lds, slot, tau, live, mem, scale, no_state,
                                                  no_mfma);
    lds_barrier();  // every gather has read the transform area
    if (live) {
#pragma unroll
      for (int c = 0; c < R; ++c)
        if ((uint32_t)(c * T + tau) < n_nodes) lds[slot * n_nodes + c * T + tau] = vals[c];
    }
    lds_barrier();  // node values complete
    // Leaf solves, element e: {node | caller position << 16, inverse-row
    // offset, mu(v)}; mu(v) = 0 marks no element.  B elements per thread at a
    // time: their records, then all MU entries of their inverse rows (the
    // table's zero padding keeps the rows' reads in bounds), are requested
    // before any is used, so the two dependent cache round trips are paid
    // once per batch.
    constexpr int B = sas_solve_batch<MU>();
    for (uint32_t e0 = tid; e0 < k; e0 += B * THREADS) {
      uint4 r[B];
#pragma unroll
      for (int i = 0; i < B; ++i) {
        const uint32_t e = e0 + i * THREADS;
        r[i] = e < k ? rec[e] : make_uint4(0u, 0u, 0u, 0u);
      }
      cplx64 w[B][MU];
#pragma unroll
      for (int i = 0; i < B; ++i)
#pragma unroll
        for (int jj = 0; jj < MU; ++jj) w[i][jj] = inv[r[i].y + jj];
#pragma unroll
      for (int i = 0; i < B; ++i) {
        const uint32_t nv = r[i].x & 0xffffu;
        double ar = 0.0, ai = 0.0;
#pragma unroll
        for (int jj = 0; jj < MU; ++jj) {
          if ((uint32_t)jj < r[i].z) {
            const float2 q = lds[jj * n_nodes + nv];
            ar = fma(w[i][jj].x, (double)q.x, fma(-w[i][jj].y, (double)q.y, ar));
            ai = fma(w[i][jj].x, (double)q.y, fma(w[i][jj].y, (double)q.x, ai));
          }
        }
        if (r[i].z != 0) res[r[i].x >> 16] = make_float2((float)ar, (float)ai);
      }
    }
    lds_barrier();
    float2* ob = out + b * (uint64_t)ld_out;
    for (uint32_t t = tid; t < k; t += THREADS) store_stream(ob + t, res[t]);
    lds_barrier();  // the next signal overwrites the LDS
  }
}

template <int S>
static bool sas_onepass_fits_s(uint32_t mu_star, uint32_t n_nodes, uint32_t k) {
  if constexpr (!sas_onepass_shape<S>()) {
    return false;
  } else {
    constexpr uint64_t SLOTS = SasFused<S>::TRANSFORM_SLOTS;
    return mu_star <= (uint32_t)SasFused<S>::Sh::SPB && (uint64_t)mu_star * n_nodes <= SLOTS &&
           (uint64_t)mu_star * n_nodes + k <= 2 * SLOTS;
  }
}

template <int S, int MU>
static hipError_t launch_sas_onepass_mu(const float2* in, int64_t ld_in, float2* out,
                                        int64_t ld_out, uint64_t batch, uint32_t mu_star,
                                        uint32_t n_nodes, uint32_t k, const float2* tw,
                                        const uint16_t* src_node, float scale, const uint4* rec,
                                        const cplx64* inv, hipStream_t stream) {
  using Sh = typename SasFused<S>::Sh;
  constexpr uint64_t SLOTS = SasFused<S>::TRANSFORM_SLOTS;
  const uint64_t used = (uint64_t)mu_star * n_nodes + k;
  const size_t lds = (size_t)(used > SLOTS ? used : SLOTS) * sizeof(float2);
  const void* kernel = (const void*)sas_onepass_kernel<S, MU>;
  static OccupancyCache cache;
  Occupancy occ;
  if (!cache.get(&occ)) {
    hipError_t e = query_occupancy(kernel, Sh::THREADS, 2 * SLOTS * sizeof(float2), &occ);
    if (e != hipSuccess) return e;
    cache.put(occ);
  }
  int per_cu_lds = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_lds, kernel, Sh::THREADS,
                                                              lds);
  if (e != hipSuccess) return e;
  uint64_t per_cu = per_cu_lds > 0 ? (uint64_t)per_cu_lds : (uint64_t)occ.per_cu;
  uint64_t grid = per_cu * (uint64_t)occ.cus;
  if (grid > batch) grid = batch;
  hipLaunchKernelGGL((sas_onepass_kernel<S, MU>), dim3((unsigned)grid), dim3(Sh::THREADS), lds,
                     stream, in, ld_in, out, ld_out, batch, mu_star, n_nodes, k, tw, src_node,
                     scale, rec, inv);
  return hipGetLastError();
}

template <int S>
static hipError_t launch_sas_onepass(const float2* in, int64_t ld_in, float2* out, int64_t ld_out,
                                     uint64_t batch, uint32_t mu_star, uint32_t n_nodes,
                                     uint32_t k, const float2* tw, const uint16_t* src_node,
                                     float scale, const uint4* rec, const cplx64* inv,
                                     hipStream_t stream) {
  if (mu_star == 2)
    return launch_sas_onepass_mu<S, 2>(in, ld_in, out, ld_out, batch, mu_star, n_nodes, k, tw,
                                       src_node, scale, rec, inv, stream);
  if (mu_star == 3)
    return launch_sas_onepass_mu<S, 3>(in, ld_in, out, ld_out, batch, mu_star, n_nodes, k, tw,
                                       src_node, scale, rec, inv, stream);
  return launch_sas_onepass_mu<S, 4>(in, ld_in, out, ld_out, batch, mu_star, n_nodes, k, tw,
                                     src_node, scale, rec, inv, stream);
}

template <int S>
static bool sas_fused_fits_s(uint32_t mu_star, uint32_t n_nodes, uint32_t k) {
  return sas_onepass_fits_s<S>(mu_star, n_nodes, k) ||
         (k <= (uint32_t)(SAS_FUSED_EPT * SasFused<S>::Sh::THREADS) &&
          SasFused<S>::lds_bytes(mu_star, n_nodes, k) <= SAS_FUSED_MAX_LDS);
}

template <int S>
static hipError_t launch_sas_fused_s(const float2* in, int64_t ld_in, float2* out, int64_t ld_out,
                                     uint64_t batch, uint32_t mu_star, uint32_t n_nodes,
                                     uint32_t k, const float2* tw, const uint16_t* src_node,
                                     float scale, const uint4* rec, const cplx64* inv,
                                     hipStream_t stream) {
  if constexpr (sas_onepass_shape<S>()) {
    if (sas_onepass_fits_s<S>(mu_star, n_nodes, k))
      return launch_sas_onepass<S>(in, ld_in, out, ld_out, batch, mu_star, n_nodes, k, tw,
                                   src_node, scale, rec, inv, stream);
  }
  using Sh = typename SasFused<S>::Sh;
  const size_t lds = SasFused<S>::lds_bytes(mu_star, n_nodes, k);
  static OccupancyCache cache;
  Occupancy occ;
  if (!cache.get(&occ)) {
    hipError_t e = query_occupancy((const void*)sas_fused_kernel<S>, Sh::THREADS,
                                   SAS_FUSED_MAX_LDS, &occ);
    if (e != hipSuccess) return e;
    cache.put(occ);
  }
  // Blocks per CU: by this plan's LDS size, and by registers (the occupancy
  // query above, at the largest LDS size, bounds it from below).
  int per_cu_regs = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu_regs, (const void*)sas_fused_kernel<S>, Sh::THREADS, lds);
  if (e != hipSuccess) return e;
  uint64_t per_cu = per_cu_regs > 0 ? (uint64_t)per_cu_regs : (uint64_t)occ.per_cu;
  uint64_t grid = per_cu * (uint64_t)occ.cus;
  if (grid > batch) grid = batch;
  hipLaunchKernelGGL(sas_fused_kernel<S>, dim3((unsigned)grid), dim3(Sh::THREADS), lds, stream,
                     in, ld_in, out, ld_out, batch, mu_star, n_nodes, k, tw, src_node, scale,
                     rec, inv);
  return hipGetLastError();
}

bool sas_fused_fits(uint32_t s, uint32_t mu_star, uint32_t n_nodes, uint32_t k) {
  if (mu_star < 2 || mu_star > 4 || n_nodes == 0 || k == 0) return false;
  switch (s) {
#define HIDFT_CASE(S) \
  case S:             \
    return sas_fused_fits_s<S>(mu_star, n_nodes, k);
    HIDFT_CASE(1) HIDFT_CASE(2) HIDFT_CASE(3) HIDFT_CASE(4) HIDFT_CASE(5) HIDFT_CASE(6)
    HIDFT_CASE(7) HIDFT_CASE(8) HIDFT_CASE(9) HIDFT_CASE(10) HIDFT_CASE(11) HIDFT_CASE(12)
    HIDFT_CASE(13)
#undef HIDFT_CASE
    default:
      return false;
  }
}

hipError_t launch_sas_fused(uint32_t s, const float2* in, int64_t ld_in, float2* out,
                            int64_t ld_out, uint64_t batch, uint32_t mu_star, uint32_t n_nodes,
                            uint32_t k, const float2* tw, const uint16_t* src_node, float scale,
                            const void* elem_rec, const void* inv, hipStream_t stream) {
  if (!sas_fused_fits(s, mu_star, n_nodes, k) || elem_rec == nullptr) return hipErrorInvalidValue;
  if (batch == 0) return hipSuccess;
  const uint4* rec = static_cast<const uint4*>(elem_rec);
  const cplx64* m = static_cast<const cplx64*>(inv);
  switch (s) {
#define HIDFT_CASE(S) \
  case S:             \
    return launch_sas_fused_s<S>(in, ld_in, out, ld_out, batch, mu_star, n_nodes, k, tw, \
                                 src_node, scale, rec, m, stream);
    HIDFT_CASE(1) HIDFT_CASE(2) HIDFT_CASE(3) HIDFT_CASE(4) HIDFT_CASE(5) HIDFT_CASE(6)
    HIDFT_CASE(7) HIDFT_CASE(8) HIDFT_CASE(9) HIDFT_CASE(10) HIDFT_CASE(11) HIDFT_CASE(12)
    HIDFT_CASE(13)
#undef HIDFT_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_sas_apply(const float2* y, uint32_t n_nodes, uint32_t mu_star, uint64_t batch,
                            uint32_t k, const uint32_t* elem_node, const uint32_t* node_first,
                            const uint32_t* node_count, const uint32_t* inv_off, const void* inv,
                            const uint32_t* elem_t, const void* elem_rec, float2* out,
                            int64_t ld_out, hipStream_t stream) {
  if (batch == 0 || k == 0) return hipSuccess;
  const cplx64* m = static_cast<const cplx64*>(inv);
  if ((uint64_t)mu_star * n_nodes + k <= (uint64_t)SAS_LDS_VALUES) {
    if (elem_rec == nullptr) return hipErrorInvalidValue;
    const uint4* rec = static_cast<const uint4*>(elem_rec);
    // Elements per thread: k / SAS_LDS_THREADS rounded up to a power of two.
    // The nodes' element counts sum to k <= mu* n_nodes, so k is at most half
    // of SAS_LDS_VALUES: at most 8 elements per thread.
    static_assert(SAS_LDS_VALUES / 2 <= 8 * SAS_LDS_THREADS, "at most 8 elements per thread");
    const uint32_t per = (k + SAS_LDS_THREADS - 1) / SAS_LDS_THREADS;
    if (per <= 1)
      return launch_sas_apply_lds_mu<1>(y, n_nodes, mu_star, batch, k, rec, m, out, ld_out, stream);
    if (per <= 2)
      return launch_sas_apply_lds_mu<2>(y, n_nodes, mu_star, batch, k, rec, m, out, ld_out, stream);
    if (per <= 4)
      return launch_sas_apply_lds_mu<4>(y, n_nodes, mu_star, batch, k, rec, m, out, ld_out, stream);
    if (per <= 8)
      return launch_sas_apply_lds_mu<8>(y, n_nodes, mu_star, batch, k, rec, m, out, ld_out, stream);
    return hipErrorInvalidValue;
  }
  const unsigned gx = (k + SAS_APPLY_THREADS - 1) / SAS_APPLY_THREADS;
  // Enough blocks along the batch to fill the device, each striding over signals.
  uint64_t gy = (4096 + gx - 1) / gx;
  if (gy > batch) gy = batch;
  if (gy > 65535) gy = 65535;
  if (gy == 0) gy = 1;
  hipLaunchKernelGGL(sas_apply_kernel, dim3(gx, (unsigned)gy), dim3(SAS_APPLY_THREADS), 0,
                     stream, y, n_nodes, mu_star, batch, k, elem_node, node_first, node_count,
                     inv_off, m, elem_t, out, ld_out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Transforms of more than 2^14 points, in passes through a workspace.
//
// The recursion splits at any level (Corollary 2).  With s = s1 + s2
// (s2 = 12 up to s = 20, then s - 9; s1 <= 9):
//  * pass 1: stages 1..s1 pair only the top s1 bits of the position a, and
//    their twiddles depend on those bits alone, so for every value of the
//    low s2 bits (a column) the 2^s1 values of the column form a transform
//    with the same s1-stage twiddles.  Up to s1 = 4 a thread takes one
//    column, in registers; above, a block takes a tile of columns through
//    two groups (stages 1..4 on the top four bits, stages 5..s1 on the rest,
//    s1 <= 8) or three (s1 = 9) with exchanges in LDS.
//  * pass 2: stages s1+1..s never mix values whose top s1 bits differ, so
//    each subtree (2^s2 consecutive positions) is a transform of 2^s2 points
//    whose stage-u' twiddles are the run of stage s1+u' starting at
//    subtree * 2^(u'-1).  The plan keeps these runs in the fused kernel's
//    table layout, one table per subtree, and the fused kernel's per-signal
//    code runs each subtree in place.  Its gather writes the subtree's
//    outputs ordered by their index t in the caller's order of J.
//  * pass 3: output chunk c (large_chunk(s) consecutive t, of the n_out <= 2^s
//    outputs kept; the last chunk may be partial) takes from each
//    subtree the contiguous run of its outputs whose t fall in the chunk,
//    puts each value at its place in LDS, scales by N/k and stores the chunk
//    in order.  Every read and write of the pass is a contiguous run; only
//    the LDS writes are scattered.
// Every stage's arithmetic is the single-pass kernel's, in the same order.
// ---------------------------------------------------------------------------
constexpr int LARGE_THREADS = 256;

template <int S1>
__global__ void __launch_bounds__(LARGE_THREADS)
large_top_kernel(const float2* __restrict__ in, int64_t ld_in, float2* __restrict__ work,
                 uint64_t batch, uint32_t s2, const float2* __restrict__ tw) {
  constexpr int R1 = 1 << S1;
  float2 w[R1 - 1];
#pragma unroll
  for (int i = 0; i < R1 - 1; ++i) w[i] = make_uniform(tw[i]);
  const uint64_t cols = 1ULL << s2;
  const uint64_t k = cols << S1;
  const uint64_t n = batch << s2;
  const uint64_t stride = (uint64_t)gridDim.x * LARGE_THREADS;
  for (uint64_t i = (uint64_t)blockIdx.x * LARGE_THREADS + threadIdx.x; i < n; i += stride) {
    const uint64_t b = i >> s2, col = i & (cols - 1);
    const float2* x = in + b * (uint64_t)ld_in + col;
    float2 v[R1];
#pragma unroll
    for (int h = 0; h < R1; ++h) v[h] = load_stream(x + (uint64_t)h * cols);
#pragma unroll
    for (int u = 1; u <= S1; ++u) {
      const int bit = S1 - u;
#pragma unroll
      for (int c = 0; c < R1; ++c) {
        if (c & (1 << bit)) continue;
        butterfly(v[c], v[c | (1 << bit)], w[(1 << (u - 1)) - 1 + (c >> (bit + 1))]);
      }
    }
    float2* y = work + b * k + col;
#pragma unroll
    for (int h = 0; h < R1; ++h) y[(uint64_t)h * cols] = v[h];
  }
}

// Columns for s1 = 5..8: a block takes COLS consecutive columns of one
// signal.  Group A: thread (g, col) holds the 16 values h = c RB + g (c <
// 16) of column col and runs stages 1..4 (the top four bits of h, uniform
// twiddles).  Group B, after an exchange in LDS: unit (c, col) holds the RB
// values h = c RB + g (g < RB) and runs stages 5..s1, whose twiddles depend
// on the bits of h above the stage's bit (the table's first 2^s1 - 1 entries,
// copied to LDS).  At s1 = 8 a block has 512 threads, so that its tile is 32
// columns wide and each of the 256 row segments it reads is 256 B (128 B with
// 256 threads: 158.6 against 155.0 us at 2^20 points).
template <int S1>
constexpr int top2_threads() { return S1 == 8 ? 512 : LARGE_THREADS; }

template <int S1, int THREADS = top2_threads<S1>()>
__global__ void __launch_bounds__(THREADS)
large_top2_kernel(const float2* __restrict__ in, int64_t ld_in, float2* __restrict__ work,
                  uint64_t batch, uint32_t s2, const float2* __restrict__ tw) {
  static_assert(S1 >= 5 && S1 <= 8, "two groups of at most four stages");
  constexpr int RB = 1 << (S1 - 4);
  constexpr int COLS = THREADS / RB;
  constexpr int H = 1 << S1;
  constexpr int PAD_H = H + 1;  // odd column stride in LDS
  __shared__ float2 L[COLS * PAD_H];
  __shared__ float2 T[H - 1];
  for (int i = threadIdx.x; i < H - 1; i += THREADS) T[i] = tw[i];
  float2 w1[15];
#pragma unroll
  for (int i = 0; i < 15; ++i) w1[i] = make_uniform(tw[i]);
  __syncthreads();
  const uint64_t cols = 1ULL << s2;
  const uint64_t k = cols << S1;
  const uint64_t tiles_per_signal = cols / COLS;
  const uint64_t tiles = batch * tiles_per_signal;
  for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const uint64_t b = tile / tiles_per_signal;
    const uint64_t col0 = (tile - b * tiles_per_signal) * COLS;
    {
      const int col = threadIdx.x % COLS, g = threadIdx.x / COLS;
      const float2* x = in + b * (uint64_t)ld_in + col0 + col;
      float2 v[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) v[c] = load_stream(x + (uint64_t)(c * RB + g) * cols);
#pragma unroll
      for (int u = 1; u <= 4; ++u) {
        const int bit = 4 - u;
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          if (c & (1 << bit)) continue;
          butterfly(v[c], v[c | (1 << bit)], w1[(1 << (u - 1)) - 1 + (c >> (bit + 1))]);
        }
      }
#pragma unroll
      for (int c = 0; c < 16; ++c) L[col * PAD_H + c * RB + g] = v[c];
    }
    lds_barrier();
    for (int unit = threadIdx.x; unit < COLS * 16; unit += THREADS) {
      const int col = unit % COLS, c = unit / COLS;
      float2 v[RB];
#pragma unroll
      for (int g = 0; g < RB; ++g) v[g] = L[col * PAD_H + c * RB + g];
#pragma unroll
      for (int u = 5; u <= S1; ++u) {
        const int bit = S1 - u;
#pragma unroll
        for (int g = 0; g < RB; ++g) {
          if (g & (1 << bit)) continue;
          const int h = c * RB + g;
          butterfly(v[g], v[g | (1 << bit)], T[(1 << (u - 1)) - 1 + (h >> (bit + 1))]);
        }
      }
      float2* y = work + b * k + col0 + col;
#pragma unroll
      for (int g = 0; g < RB; ++g) y[(uint64_t)(c * RB + g) * cols] = v[g];
    }
    lds_barrier();  // the next tile overwrites L
  }
}

// Columns for s1 = 9, in three groups so that a thread holds 16 values: a
// block of 512 threads takes 16 columns (h = row of the column, 0..511).
//  * group A, stages 1..4 (bits 8..5 of h, uniform twiddles): thread (g, col)
//    holds h = c * 32 + g, c < 16;
//  * group B, stages 5..8 (bits 4..1), after an exchange in LDS: unit
//    (hi, b0, col) holds h = hi * 32 + c * 2 + b0, c < 16;
//  * group C, stage 9 (bit 0), after another exchange: each thread takes 8
//    pairs (h, h + 1) and stores both.  Lanes l and l ^ 16 of group B hold
//    rows h and h ^ 1 of one column; swapping their values through lane
//    shuffles instead of this exchange made the pass 3-7 us slower (its
//    adjoint 0-2 us).
// Twiddles of stages 5..9 come from the table's first 511 entries, copied to
// LDS.  A second group of five stages (32 values per thread) would need about
// 210 registers and one block per CU.
constexpr int TOP3_S1 = 9;
constexpr int TOP3_THREADS = 512;
constexpr int TOP3_COLS = 16;

__global__ void __launch_bounds__(TOP3_THREADS, 4)
large_top3_kernel(const float2* __restrict__ in, int64_t ld_in, float2* __restrict__ work,
                  uint64_t batch, uint32_t s2, const float2* __restrict__ tw) {
  constexpr int H = 1 << TOP3_S1, PAD_H = H + 1, COLS = TOP3_COLS, THREADS = TOP3_THREADS;
  static_assert(COLS * 32 == THREADS, "one thread per (g, col)");
  __shared__ float2 L[COLS * PAD_H];
  __shared__ float2 T[H - 1];
  for (int i = threadIdx.x; i < H - 1; i += THREADS) T[i] = tw[i];
  float2 w1[15];
#pragma unroll
  for (int i = 0; i < 15; ++i) w1[i] = make_uniform(tw[i]);
  __syncthreads();
  const uint64_t cols = 1ULL << s2;
  const uint64_t k = cols << TOP3_S1;
  const uint64_t tiles_per_signal = cols / COLS;
  const uint64_t tiles = batch * tiles_per_signal;
  const int tid = (int)threadIdx.x;
  for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const uint64_t b = tile / tiles_per_signal;
    const uint64_t col0 = (tile - b * tiles_per_signal) * COLS;
    {  // group A
      const int col = tid % COLS, g = tid / COLS;
      const float2* x = in + b * (uint64_t)ld_in + col0 + col;
      float2 v[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) v[c] = load_stream(x + (uint64_t)(c * 32 + g) * cols);
#pragma unroll
      for (int u = 1; u <= 4; ++u) {
        const int bit = 4 - u;
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          if (c & (1 << bit)) continue;
          butterfly(v[c], v[c | (1 << bit)], w1[(1 << (u - 1)) - 1 + (c >> (bit + 1))]);
        }
      }
#pragma unroll
      for (int c = 0; c < 16; ++c) L[col * PAD_H + c * 32 + g] = v[c];
    }
    lds_barrier();
    {  // group B
      const int col = tid % COLS, hb = tid / COLS;  // hb = hi * 2 + b0
      const int hi = hb >> 1, b0 = hb & 1;
      float2 v[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) v[c] = L[col * PAD_H + hi * 32 + c * 2 + b0];
#pragma unroll
      for (int u = 5; u <= 8; ++u) {
        const int bit = 8 - u;  // of c; bit + 1 of h
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          if (c & (1 << bit)) continue;
          const int h = hi * 32 + c * 2 + b0;
          butterfly(v[c], v[c | (1 << bit)], T[(1 << (u - 1)) - 1 + (h >> (bit + 2))]);
        }
      }
#pragma unroll
      for (int c = 0; c < 16; ++c) L[col * PAD_H + hi * 32 + c * 2 + b0] = v[c];
    }
    lds_barrier();
    {  // group C: stage 9 on the pairs (h, h + 1), h even
      float2* y = work + b * k + col0;
#pragma unroll 2
      for (int i = 0; i < 8; ++i) {
        const int p = tid + i * THREADS;  // pair p: column p % 16, rows 2 (p / 16) + {0, 1}
        const int col = p % COLS, h = 2 * (p / COLS);
        float2 a = L[col * PAD_H + h], c = L[col * PAD_H + h + 1];
        butterfly(a, c, T[(1 << (TOP3_S1 - 1)) - 1 + (h >> 1)]);
        y[(uint64_t)h * cols + col] = a;
        y[(uint64_t)(h + 1) * cols + col] = c;
      }
    }
    lds_barrier();  // the next tile overwrites L
  }
}

// A subtree's transform: its own twiddle and gather tables, outputs stored
// over its inputs.
struct SubtreeMem {
  const float2* tw;
  const uint16_t* src;
  float2* out;
  __device__ __forceinline__ float2 tw_at(int uni, int lane) const { return tw[uni + lane]; }
  __device__ __forceinline__ int src_at(int uni, int lane) const { return src[uni + lane]; }
  __device__ __forceinline__ void put(int uni, int lane, float2 x) const { out[uni + lane] = x; }
};

// Subtree units.  Each subtree reads its own twiddle and gather tables (10 B
// per point, as much as its data) from the L2 of the XCD it runs on, and
// blocks are dispatched to the eight XCDs in turn (block g to XCD g % 8).  In
// signal-major order (unit g = signal * 2^s1 + subtree) an XCD serves 2^s1 / 8
// subtrees' tables at once: 1.3 MB at s1 = 8 (2^12-point subtrees), which
// fits its 4 MB L2 beside the streamed rows, but 2.6 and 5.2 MB at s1 = 9.
// There block g takes subtree 8 (j / batch) + g % 8 of signal j % batch,
// j = g / 8, so the batch's copies of one subtree run back to back on one XCD
// and read its tables from that L2: 2^21 points 167 -> 159 us, 2^22 183 ->
// 178 us.  Below s1 = 9 that order made the passes 5-12 us slower (the
// blocks in flight read rows of many signals instead of consecutive rows).
// A bijection on [0, units) since 8 divides 2^s1.
__device__ __forceinline__ uint64_t subtree_unit(uint64_t g, uint32_t s1, uint64_t units) {
  if (s1 < 9) return g;
  const uint64_t batch = units >> s1, j = g >> 3, m = j / batch;
  return ((j - m * batch) << s1) + (g & 7) + 8 * m;
}

template <int S2, int SCHED>
__global__ void __launch_bounds__((FusedShape<S2, SCHED, 4>::THREADS))
large_sub_kernel(float2* __restrict__ work, uint64_t first, uint64_t units, uint32_t s1,
                 const float2* __restrict__ tw2, const uint16_t* __restrict__ src2) {
  using Sh = FusedShape<S2, SCHED, 4>;
  static_assert(Sh::SPB == 1 && Sh::THREADS == Sh::T, "one subtree per block");
  constexpr int R = Sh::R, T = Sh::T;
  constexpr uint64_t K2 = 1ULL << S2;
  extern __shared__ float2 lds[];
  const uint64_t g = first + blockIdx.x;
  if (g >= units) return;  // uniform over the block
  const uint64_t unit = subtree_unit(g, s1, units);
  const uint64_t sub = unit & ((1ULL << s1) - 1);
  float2* row = work + unit * K2;  // unit = signal * 2^s1 + subtree
  float2 v[R];
  __builtin_amdgcn_s_setprio(2);
  load_row<R, T, false>(v, row, (uint32_t)K2);
  __builtin_amdgcn_s_setprio(0);
  const SubtreeMem mem{tw2 + sub * (K2 - 1), src2 + sub * K2, row};
  ThreadState<S2, SCHED, 4> unused;
  const MfmaOps<PREC_FP32> no_mfma;
  transform_signal<S2, SCHED, 4, PREC_FP32, false>(v, lds, 0, (int)threadIdx.x, true, mem, 1.0f,
                                                    unused, no_mfma);
}

// Placement of chunk c (outputs t in [c * CHUNK, ...)): src3[t] is the
// output's index in the signal's workspace row (its subtree's run), dest3[t]
// its slot in the chunk.  A whole chunk gives each thread LARGE_EPT outputs:
// all of its table reads are issued first, then all of its row reads (through
// a buffer descriptor, a 32-bit offset each), so that every thread keeps
// LARGE_EPT reads in flight.  A chunk takes one run from each of the 2^s1
// subtrees, CHUNK / 2^s1 outputs on average: chunks of 4096 (256 threads,
// 32 KB of LDS) up to s1 = 6, of 16384 (1024 threads, 128 KB) above.
constexpr int LARGE_EPT = 16;

// Chunk units in XCD order.  A chunk's run from a subtree starts anywhere in
// a 128-byte line, so the lines at a run's two ends are shared with the
// neighbouring chunks' runs; blocks go to the eight XCDs in turn (block g to
// XCD g % 8), which puts neighbouring chunks on different XCDs and moves
// each shared line through two L2s.  In every full round of the grid, block
// g takes unit (g % 8) * (grid / 8) + g / 8 of the round instead, so that
// each XCD holds a contiguous range of chunks; the last, partial round keeps
// the plain order.  A bijection on [0, units) for a grid that 8 divides.
// Used at s1 = 9 (runs of 32 outputs), where it took the forward pass
// sequence at 2^22 points from 178 to 167 us (2^21: 160 -> 157 us) and the
// inverse at 2^22 from 171 to 166 us (2^21: 1.7 us slower); at s1 <= 8 the
// forward was 8-10 us slower with it.
__device__ __forceinline__ uint64_t chunk_unit(uint64_t u, uint64_t grid, uint64_t units,
                                               uint32_t xcd_order) {
  const uint64_t round = u / grid, g = u - round * grid;
  if (!xcd_order || grid % 8 != 0 || (round + 1) * grid > units) return u;
  return round * grid + (g % 8) * (grid / 8) + g / 8;
}
template <int CHUNK>
constexpr int place_threads() {
  static_assert(CHUNK % LARGE_EPT == 0 && CHUNK / LARGE_EPT <= 1024 && CHUNK <= 65536 &&
                    CHUNK * 8 <= 128 * 1024,
                "whole chunks per block, 16-bit places, the chunk in LDS");
  return CHUNK / LARGE_EPT;
}

template <int CHUNK>
__global__ void __launch_bounds__(place_threads<CHUNK>())
large_place_kernel(const float2* __restrict__ work, float2* __restrict__ out, int64_t ld_out,
                   uint64_t batch, uint32_t s, uint64_t n_out, const uint32_t* __restrict__ src3,
                   const uint16_t* __restrict__ dest3, float scale, uint32_t xcd_order) {
  constexpr int THREADS = place_threads<CHUNK>();
  __shared__ float2 chunk[CHUNK];
  const uint64_t k = 1ULL << s;
  const uint64_t chunks = (n_out + CHUNK - 1) / CHUNK;
  const int tid = (int)threadIdx.x;
  for (uint64_t u = blockIdx.x; u < batch * chunks; u += gridDim.x) {
    const uint64_t unit = chunk_unit(u, gridDim.x, batch * chunks, xcd_order);
    const uint64_t b = unit / chunks, c = unit - b * chunks;
    const uint32_t count =
        (uint32_t)(n_out - c * CHUNK < (uint64_t)CHUNK ? n_out - c * CHUNK : (uint64_t)CHUNK);
    const float2* w = work + b * k;
    const uint32_t* s3 = src3 + c * CHUNK;
    const uint16_t* d3 = dest3 + c * CHUNK;
    if (count == (uint32_t)CHUNK) {
      const __amdgpu_buffer_rsrc_t row = make_rsrc(w, (uint32_t)(k * sizeof(float2)));
      uint32_t si[LARGE_EPT], di[LARGE_EPT];
#pragma unroll
      for (int i = 0; i < LARGE_EPT; ++i) {
        si[i] = s3[tid + i * THREADS];
        di[i] = d3[tid + i * THREADS];
      }
      float2 x[LARGE_EPT];
#pragma unroll
      for (int i = 0; i < LARGE_EPT; ++i)
        x[i] = __builtin_bit_cast(
            float2, __builtin_amdgcn_raw_buffer_load_b64(row, (int)(si[i] * sizeof(float2)), 0, 0));
#pragma unroll
      for (int i = 0; i < LARGE_EPT; ++i) chunk[di[i]] = make_float2(x[i].x * scale, x[i].y * scale);
    } else {
      for (uint32_t e = tid; e < count; e += THREADS) {
        const float2 x = w[s3[e]];
        chunk[d3[e]] = make_float2(x.x * scale, x.y * scale);
      }
    }
    lds_barrier();
    float2* o = out + b * (uint64_t)ld_out + c * CHUNK;
    for (uint32_t e = tid; e < count; e += THREADS) store_stream(o + e, chunk[e]);
    lds_barrier();  // the next unit overwrites the chunk
  }
}

// s2: 12 up to 2^20 points (s1 <= 8), then s - 9 (s1 = 9, the three-group
// column kernel): 2^21 points as 9 + 12 rather than 8 + 13 took the forward
// pass sequence from 163 to 159 us and the inverse from 172 to 164 us.
uint32_t large_split(uint32_t s) { return s > 20 ? s - TOP3_S1 : 12; }
uint32_t large_chunk(uint32_t s) { return s - large_split(s) >= 7 ? 16384u : 4096u; }

static hipError_t stream_grid(uint64_t threads, unsigned* grid) {
  static OccupancyCache cache;
  Occupancy occ;
  if (!cache.get(&occ)) {
    int dev = 0, cus = 0;
    hipError_t e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) !=
        hipSuccess)
      return e;
    occ.cus = cus > 0 ? cus : 1;
    occ.per_cu = 8;
    cache.put(occ);
  }
  const uint64_t want = (threads + LARGE_THREADS - 1) / LARGE_THREADS;
  const uint64_t cap = (uint64_t)occ.per_cu * occ.cus;
  *grid = (unsigned)(want < cap ? want : cap);
  return hipSuccess;
}

// Grid of a placement kernel: the blocks that are resident at once (by the
// chunk's LDS), at most one per chunk.
static hipError_t place_grid(const void* kernel, int threads, OccupancyCache& cache,
                             uint64_t units, unsigned* grid) {
  Occupancy occ;
  if (!cache.get(&occ)) {
    hipError_t e = query_occupancy(kernel, threads, 0, &occ);
    if (e != hipSuccess) return e;
    cache.put(occ);
  }
  const uint64_t cap = (uint64_t)(occ.per_cu > 0 ? occ.per_cu : 1) * (uint64_t)occ.cus;
  *grid = (unsigned)(units < cap ? units : cap);
  return hipSuccess;
}

template <int CHUNK>
static hipError_t launch_place(const float2* work, float2* out, int64_t ld_out, uint64_t batch,
                               uint32_t s, uint64_t n_out, const uint32_t* src3,
                               const uint16_t* dest3, float scale, hipStream_t stream) {
  constexpr int THREADS = place_threads<CHUNK>();
  static OccupancyCache cache;
  unsigned grid = 0;
  hipError_t e = place_grid((const void*)large_place_kernel<CHUNK>, THREADS, cache,
                            batch * ((n_out + CHUNK - 1) / CHUNK), &grid);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(large_place_kernel<CHUNK>, dim3(grid), dim3(THREADS), 0, stream, work, out,
                     ld_out, batch, s, n_out, src3, dest3, scale,
                     (uint32_t)(s - large_split(s) >= TOP3_S1));
  return hipGetLastError();
}

// The two-group column kernel: the blocks resident at once, at most one per
// tile of THREADS / 2^(s1 - 4) columns.
template <int S1>
static hipError_t launch_top2(const float2* in, int64_t ld_in, float2* work, uint64_t batch,
                              uint32_t s2, const float2* tw, hipStream_t stream) {
  constexpr int THREADS = top2_threads<S1>();
  constexpr uint64_t COLS = (uint64_t)THREADS >> (S1 - 4);
  static OccupancyCache cache;
  Occupancy occ;
  if (!cache.get(&occ)) {
    hipError_t e = query_occupancy((const void*)large_top2_kernel<S1>, THREADS, 0, &occ);
    if (e != hipSuccess) return e;
    cache.put(occ);
  }
  const uint64_t tiles = (batch << s2) / COLS;
  const uint64_t cap = (uint64_t)occ.per_cu * (uint64_t)occ.cus;
  const unsigned grid = (unsigned)(tiles < cap ? tiles : cap);
  hipLaunchKernelGGL(large_top2_kernel<S1>, dim3(grid), dim3(THREADS), 0, stream, in, ld_in,
                     work, batch, s2, tw);
  return hipGetLastError();
}

// The three-group column kernel (s1 = 9), or its adjoint: the blocks
// resident at once, at most one per tile of 16 columns.
static hipError_t top3_grid(const void* kernel, int threads, int cols, OccupancyCache& cache,
                            uint64_t batch, uint32_t s2, unsigned* grid) {
  Occupancy occ;
  if (!cache.get(&occ)) {
    hipError_t e = query_occupancy(kernel, threads, 0, &occ);
    if (e != hipSuccess) return e;
    cache.put(occ);
  }
  const uint64_t tiles = (batch << s2) / (uint64_t)cols;
  const uint64_t cap = (uint64_t)occ.per_cu * (uint64_t)occ.cus;
  *grid = (unsigned)(tiles < cap ? tiles : cap);
  return hipSuccess;
}

template <int S2, int SCHED>
static hipError_t launch_large_sub(float2* work, uint64_t units, uint32_t s1, const float2* tw2,
                                   const uint16_t* src2, hipStream_t stream) {
  using Sh = FusedShape<S2, SCHED, 4>;
  static OccupancyCache cache;
  Occupancy occ;
  if (!cache.get(&occ)) {
    hipError_t e = query_occupancy((const void*)large_sub_kernel<S2, SCHED>, Sh::THREADS,
                                   Sh::LDS_BYTES, &occ);
    if (e != hipSuccess) return e;
    cache.put(occ);
  }
  const uint64_t chunk = 0x7fffffffULL;
  for (uint64_t first = 0; first < units; first += chunk) {
    const uint64_t n = units - first < chunk ? units - first : chunk;
    hipLaunchKernelGGL((large_sub_kernel<S2, SCHED>), dim3((unsigned)n), dim3(Sh::THREADS),
                       Sh::LDS_BYTES, stream, work, first, units, s1, tw2, src2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_large(uint32_t s, const float2* in, int64_t ld_in, float2* out,
                        int64_t ld_out, uint64_t batch, float2* work, const float2* tw,
                        const uint16_t* src2, const uint32_t* src3, const uint16_t* dest3,
                        float scale, hipStream_t stream, uint64_t n_out) {
  if (batch == 0) return hipSuccess;
  if (s <= HIDFT_MAX_LOG2_K_DEVICE || s > HIDFT_MAX_LOG2_K_LARGE) return hipErrorInvalidValue;
  const uint32_t s2 = large_split(s), s1 = s - s2;
  const uint64_t k = 1ULL << s;
  if (batch > (~0ULL >> (s + 1))) return hipErrorInvalidValue;
  if (n_out == 0) n_out = k;
  if (n_out > k) return hipErrorInvalidValue;
  unsigned grid = 0;
  hipError_t e = stream_grid(batch << s2, &grid);
  if (e != hipSuccess) return e;
  switch (s1) {
#define HIDFT_TOP(S1)                                                                       \
  case S1:                                                                                  \
    hipLaunchKernelGGL(large_top_kernel<S1>, dim3(grid), dim3(LARGE_THREADS), 0, stream, in, \
                       ld_in, work, batch, s2, tw);                                         \
    break;
#define HIDFT_TOP2(S1)                                                                      \
  case S1:                                                                                  \
    if ((e = launch_top2<S1>(in, ld_in, work, batch, s2, tw, stream)) != hipSuccess) return e; \
    break;
    HIDFT_TOP(1) HIDFT_TOP(2) HIDFT_TOP(3) HIDFT_TOP(4)
    HIDFT_TOP2(5) HIDFT_TOP2(6) HIDFT_TOP2(7) HIDFT_TOP2(8)
#undef HIDFT_TOP
#undef HIDFT_TOP2
    case TOP3_S1: {
      static OccupancyCache cache3;
      unsigned grid3 = 0;
      if ((e = top3_grid((const void*)large_top3_kernel, TOP3_THREADS, TOP3_COLS, cache3, batch,
                         s2, &grid3)) !=
          hipSuccess)
        return e;
      hipLaunchKernelGGL(large_top3_kernel, dim3(grid3), dim3(TOP3_THREADS), 0, stream, in,
                         ld_in, work, batch, s2, tw);
      break;
    }
    default:
      return hipErrorInvalidValue;
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const float2* tw2 = tw + ((1u << s1) - 1);
  const uint64_t units = batch << s1;
  switch (s2) {
    case 12: e = launch_large_sub<12, SCHED_SHORT_LAST>(work, units, s1, tw2, src2, stream); break;
    case 13: e = launch_large_sub<13, SCHED_SHORT_LAST>(work, units, s1, tw2, src2, stream); break;
    case 14: e = launch_large_sub<14, SCHED_SHORT_LAST>(work, units, s1, tw2, src2, stream); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if (large_chunk(s) == 4096)
    return launch_place<4096>(work, out, ld_out, batch, s, n_out, src3, dest3, scale, stream);
  return launch_place<16384>(work, out, ld_out, batch, s, n_out, src3, dest3, scale, stream);
}

// ---------------------------------------------------------------------------
// Inverse map above 2^14 points: the adjoint of the three passes, in reverse.
//  * placement^H: chunk c of the coefficients (large_chunk(s) consecutive t) is
//    read in order into LDS and written to the subtree runs of the workspace
//    (the forward placement's tables, read the other way);
//  * subtrees^H: each subtree runs the inverse kernel's per-signal code
//    (inverse_signal) with its own twiddle and gather tables, in place;
//  * columns^H: the adjoint of stages s1..1 per column, scaled by `scale`
//    (1/N), stored as the samples in ascending order of I_r.
// ---------------------------------------------------------------------------
template <int CHUNK>
__global__ void __launch_bounds__(place_threads<CHUNK>())
large_unplace_kernel(const float2* __restrict__ coefs, int64_t ld_in, float2* __restrict__ work,
                     uint64_t batch, uint32_t s, const uint32_t* __restrict__ src3,
                     const uint16_t* __restrict__ dest3, uint32_t xcd_order) {
  constexpr int THREADS = place_threads<CHUNK>();
  __shared__ float2 chunk[CHUNK];
  const uint64_t k = 1ULL << s;
  const uint64_t chunks = k / CHUNK;
  const int tid = (int)threadIdx.x;
  for (uint64_t u = blockIdx.x; u < batch * chunks; u += gridDim.x) {
    const uint64_t unit = chunk_unit(u, gridDim.x, batch * chunks, xcd_order);
    const uint64_t b = unit / chunks, c = unit - b * chunks;
    const float2* x = coefs + b * (uint64_t)ld_in + c * CHUNK;
    const uint32_t* s3 = src3 + c * CHUNK;
    const uint16_t* d3 = dest3 + c * CHUNK;
    uint32_t si[LARGE_EPT], di[LARGE_EPT];
#pragma unroll
    for (int i = 0; i < LARGE_EPT; ++i) {
      chunk[tid + i * THREADS] = load_stream(x + tid + i * THREADS);
      si[i] = s3[tid + i * THREADS];
      di[i] = d3[tid + i * THREADS];
    }
    lds_barrier();
    const __amdgpu_buffer_rsrc_t row = make_rsrc(work + b * k, (uint32_t)(k * sizeof(float2)));
#pragma unroll
    for (int i = 0; i < LARGE_EPT; ++i)
      __builtin_amdgcn_raw_buffer_store_b64(
          __builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, chunk[di[i]]), row,
          (int)(si[i] * sizeof(float2)), 0, 0);
    lds_barrier();  // the next unit overwrites the chunk
  }
}

template <int S2, int SCHED>
__global__ void __launch_bounds__((FusedShape<S2, SCHED, 4>::THREADS))
large_sub_inv_kernel(float2* __restrict__ work, uint64_t first, uint64_t units, uint32_t s1,
                     const float2* __restrict__ tw2, const uint16_t* __restrict__ src2) {
  using Sh = FusedShape<S2, SCHED, 4>;
  static_assert(Sh::SPB == 1 && Sh::THREADS == Sh::T, "one subtree per block");
  constexpr int R = Sh::R, T = Sh::T;
  constexpr uint64_t K2 = 1ULL << S2;
  extern __shared__ float2 lds[];
  const uint64_t g = first + blockIdx.x;
  if (g >= units) return;  // uniform over the block
  const uint64_t unit = subtree_unit(g, s1, units);
  const uint64_t sub = unit & ((1ULL << s1) - 1);
  float2* row = work + unit * K2;
  const int tau = (int)threadIdx.x;
  AdjointMem<R, T> mem;
  mem.tw = tw2 + sub * (K2 - 1);
  mem.read_places(src2 + sub * K2, tau);  // ahead of the row
  mem.template read_first_twiddles<S2, SCHED>(tau);
  float2 v[R];
  __builtin_amdgcn_s_setprio(2);
  load_row<R, T, false>(v, row, (uint32_t)K2);
  __builtin_amdgcn_s_setprio(0);
  ThreadState<S2, SCHED, 4> unused;
  inverse_signal<S2, SCHED, false>(v, lds, tau, mem, unused);
#pragma unroll
  for (int c = 0; c < R; ++c) row[c * T + tau] = v[c];
}

template <int S1>
__global__ void __launch_bounds__(LARGE_THREADS)
large_top_inv_kernel(const float2* __restrict__ work, float2* __restrict__ out, int64_t ld_out,
                     uint64_t batch, uint32_t s2, const float2* __restrict__ tw, float scale) {
  constexpr int R1 = 1 << S1;
  float2 w[R1 - 1];
#pragma unroll
  for (int i = 0; i < R1 - 1; ++i) w[i] = make_uniform(tw[i]);
  const uint64_t cols = 1ULL << s2;
  const uint64_t k = cols << S1;
  const uint64_t n = batch << s2;
  const uint64_t stride = (uint64_t)gridDim.x * LARGE_THREADS;
  for (uint64_t i = (uint64_t)blockIdx.x * LARGE_THREADS + threadIdx.x; i < n; i += stride) {
    const uint64_t b = i >> s2, col = i & (cols - 1);
    const float2* x = work + b * k + col;
    float2 v[R1];
#pragma unroll
    for (int h = 0; h < R1; ++h) v[h] = x[(uint64_t)h * cols];
#pragma unroll
    for (int u = S1; u >= 1; --u) {
      const int bit = S1 - u;
#pragma unroll
      for (int c = 0; c < R1; ++c) {
        if (c & (1 << bit)) continue;
        butterfly_adj(v[c], v[c | (1 << bit)], w[(1 << (u - 1)) - 1 + (c >> (bit + 1))]);
      }
    }
    float2* y = out + b * (uint64_t)ld_out + col;
#pragma unroll
    for (int h = 0; h < R1; ++h)
      store_stream(y + (uint64_t)h * cols, make_float2(v[h].x * scale, v[h].y * scale));
  }
}

// The adjoint of large_top2_kernel: group B's stages s1..5 first, then the
// exchange, then group A's stages 4..1.
template <int S1>
__global__ void __launch_bounds__(LARGE_THREADS)
large_top2_inv_kernel(const float2* __restrict__ work, float2* __restrict__ out, int64_t ld_out,
                      uint64_t batch, uint32_t s2, const float2* __restrict__ tw, float scale) {
  static_assert(S1 >= 5 && S1 <= 8, "two groups of at most four stages");
  constexpr int RB = 1 << (S1 - 4);
  constexpr int COLS = LARGE_THREADS / RB;
  constexpr int H = 1 << S1;
  constexpr int PAD_H = H + 1;
  __shared__ float2 L[COLS * PAD_H];
  __shared__ float2 T[H - 1];
  for (int i = threadIdx.x; i < H - 1; i += LARGE_THREADS) T[i] = tw[i];
  float2 w1[15];
#pragma unroll
  for (int i = 0; i < 15; ++i) w1[i] = make_uniform(tw[i]);
  __syncthreads();
  const uint64_t cols = 1ULL << s2;
  const uint64_t k = cols << S1;
  const uint64_t tiles_per_signal = cols / COLS;
  const uint64_t tiles = batch * tiles_per_signal;
  for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const uint64_t b = tile / tiles_per_signal;
    const uint64_t col0 = (tile - b * tiles_per_signal) * COLS;
    for (int unit = threadIdx.x; unit < COLS * 16; unit += LARGE_THREADS) {
      const int col = unit % COLS, c = unit / COLS;
      const float2* x = work + b * k + col0 + col;
      float2 v[RB];
#pragma unroll
      for (int g = 0; g < RB; ++g) v[g] = x[(uint64_t)(c * RB + g) * cols];
#pragma unroll
      for (int u = S1; u >= 5; --u) {
        const int bit = S1 - u;
#pragma unroll
        for (int g = 0; g < RB; ++g) {
          if (g & (1 << bit)) continue;
          const int h = c * RB + g;
          butterfly_adj(v[g], v[g | (1 << bit)], T[(1 << (u - 1)) - 1 + (h >> (bit + 1))]);
        }
      }
#pragma unroll
      for (int g = 0; g < RB; ++g) L[col * PAD_H + c * RB + g] = v[g];
    }
    lds_barrier();
    {
      const int col = threadIdx.x % COLS, g = threadIdx.x / COLS;
      float2 v[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) v[c] = L[col * PAD_H + c * RB + g];
#pragma unroll
      for (int u = 4; u >= 1; --u) {
        const int bit = 4 - u;
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          if (c & (1 << bit)) continue;
          butterfly_adj(v[c], v[c | (1 << bit)], w1[(1 << (u - 1)) - 1 + (c >> (bit + 1))]);
        }
      }
      float2* y = out + b * (uint64_t)ld_out + col0 + col;
#pragma unroll
      for (int c = 0; c < 16; ++c)
        store_stream(y + (uint64_t)(c * RB + g) * cols,
                     make_float2(v[c].x * scale, v[c].y * scale));
    }
    lds_barrier();  // the next tile overwrites L
  }
}

template <int CHUNK>
static hipError_t launch_unplace(const float2* coefs, int64_t ld_in, float2* work, uint64_t batch,
                                 uint32_t s, const uint32_t* src3, const uint16_t* dest3,
                                 hipStream_t stream) {
  constexpr int THREADS = place_threads<CHUNK>();
  static OccupancyCache cache;
  unsigned grid = 0;
  hipError_t e = place_grid((const void*)large_unplace_kernel<CHUNK>, THREADS, cache,
                            batch * ((1ULL << s) / CHUNK), &grid);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(large_unplace_kernel<CHUNK>, dim3(grid), dim3(THREADS), 0, stream, coefs,
                     ld_in, work, batch, s, src3, dest3,
                     (uint32_t)(s - large_split(s) >= TOP3_S1));
  return hipGetLastError();
}

// The adjoint of large_top3_kernel: stage 9 on the pairs first, then group
// B's stages 8..5, then group A's stages 4..1, scaled by `scale`.  Its tiles
// are 32 columns wide (1024 threads, 135 KB of LDS, one block per CU): 2-3 us
// less per pass than 16 columns at 2^21 and 2^22 points, where the forward
// kernel was 4-5 us slower with them.
constexpr int TOP3_INV_THREADS = 1024;
constexpr int TOP3_INV_COLS = 32;
__global__ void __launch_bounds__(TOP3_INV_THREADS, 4)
large_top3_inv_kernel(const float2* __restrict__ work, float2* __restrict__ out, int64_t ld_out,
                      uint64_t batch, uint32_t s2, const float2* __restrict__ tw, float scale) {
  constexpr int H = 1 << TOP3_S1, PAD_H = H + 1;
  constexpr int COLS = TOP3_INV_COLS, THREADS = TOP3_INV_THREADS;
  static_assert(COLS * 32 == THREADS, "one thread per (g, col)");
  __shared__ float2 L[COLS * PAD_H];
  __shared__ float2 T[H - 1];
  for (int i = threadIdx.x; i < H - 1; i += THREADS) T[i] = tw[i];
  float2 w1[15];
#pragma unroll
  for (int i = 0; i < 15; ++i) w1[i] = make_uniform(tw[i]);
  __syncthreads();
  const uint64_t cols = 1ULL << s2;
  const uint64_t k = cols << TOP3_S1;
  const uint64_t tiles_per_signal = cols / COLS;
  const uint64_t tiles = batch * tiles_per_signal;
  const int tid = (int)threadIdx.x;
  for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const uint64_t b = tile / tiles_per_signal;
    const uint64_t col0 = (tile - b * tiles_per_signal) * COLS;
    {  // stage 9 on the pairs (h, h + 1), h even
      const float2* x = work + b * k + col0;
#pragma unroll 4
      for (int i = 0; i < 8; ++i) {
        const int p = tid + i * THREADS;
        const int col = p % COLS, h = 2 * (p / COLS);
        float2 a = x[(uint64_t)h * cols + col], c = x[(uint64_t)(h + 1) * cols + col];
        butterfly_adj(a, c, T[(1 << (TOP3_S1 - 1)) - 1 + (h >> 1)]);
        L[col * PAD_H + h] = a;
        L[col * PAD_H + h + 1] = c;
      }
    }
    lds_barrier();
    {  // group B^H: stages 8..5
      const int col = tid % COLS, hb = tid / COLS;
      const int hi = hb >> 1, b0 = hb & 1;
      float2 v[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) v[c] = L[col * PAD_H + hi * 32 + c * 2 + b0];
#pragma unroll
      for (int u = 8; u >= 5; --u) {
        const int bit = 8 - u;
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          if (c & (1 << bit)) continue;
          const int h = hi * 32 + c * 2 + b0;
          butterfly_adj(v[c], v[c | (1 << bit)], T[(1 << (u - 1)) - 1 + (h >> (bit + 2))]);
        }
      }
#pragma unroll
      for (int c = 0; c < 16; ++c) L[col * PAD_H + hi * 32 + c * 2 + b0] = v[c];
    }
    lds_barrier();
    {  // group A^H: stages 4..1, then the scaled store
      const int col = tid % COLS, g = tid / COLS;
      float2 v[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) v[c] = L[col * PAD_H + c * 32 + g];
#pragma unroll
      for (int u = 4; u >= 1; --u) {
        const int bit = 4 - u;
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          if (c & (1 << bit)) continue;
          butterfly_adj(v[c], v[c | (1 << bit)], w1[(1 << (u - 1)) - 1 + (c >> (bit + 1))]);
        }
      }
      float2* y = out + b * (uint64_t)ld_out + col0 + col;
#pragma unroll
      for (int c = 0; c < 16; ++c)
        store_stream(y + (uint64_t)(c * 32 + g) * cols,
                     make_float2(v[c].x * scale, v[c].y * scale));
    }
    lds_barrier();  // the next tile overwrites L
  }
}

template <int S2, int SCHED>
static hipError_t launch_large_sub_inv(float2* work, uint64_t units, uint32_t s1,
                                       const float2* tw2, const uint16_t* src2,
                                       hipStream_t stream) {
  using Sh = FusedShape<S2, SCHED, 4>;
  static OccupancyCache cache;
  Occupancy occ;
  if (!cache.get(&occ)) {
    hipError_t e = query_occupancy((const void*)large_sub_inv_kernel<S2, SCHED>, Sh::THREADS,
                                   Sh::LDS_BYTES, &occ);
    if (e != hipSuccess) return e;
    cache.put(occ);
  }
  const uint64_t chunk = 0x7fffffffULL;
  for (uint64_t first = 0; first < units; first += chunk) {
    const uint64_t n = units - first < chunk ? units - first : chunk;
    hipLaunchKernelGGL((large_sub_inv_kernel<S2, SCHED>), dim3((unsigned)n), dim3(Sh::THREADS),
                       Sh::LDS_BYTES, stream, work, first, units, s1, tw2, src2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_large_inverse(uint32_t s, const float2* coefs, int64_t ld_in, float2* out,
                                int64_t ld_out, uint64_t batch, float2* work, const float2* tw,
                                const uint16_t* src2, const uint32_t* src3,
                                const uint16_t* dest3, float scale, hipStream_t stream) {
  if (batch == 0) return hipSuccess;
  if (s <= HIDFT_MAX_LOG2_K_DEVICE || s > HIDFT_MAX_LOG2_K_LARGE) return hipErrorInvalidValue;
  const uint32_t s2 = large_split(s), s1 = s - s2;
  if (batch > (~0ULL >> (s + 1))) return hipErrorInvalidValue;
  unsigned grid = 0;
  hipError_t e = large_chunk(s) == 4096
                     ? launch_unplace<4096>(coefs, ld_in, work, batch, s, src3, dest3, stream)
                     : launch_unplace<16384>(coefs, ld_in, work, batch, s, src3, dest3, stream);
  if (e != hipSuccess) return e;
  const float2* tw2 = tw + ((1u << s1) - 1);
  const uint64_t units = batch << s1;
  switch (s2) {
    case 12: e = launch_large_sub_inv<12, SCHED_SHORT_LAST>(work, units, s1, tw2, src2, stream); break;
    case 13: e = launch_large_sub_inv<13, SCHED_SHORT_LAST>(work, units, s1, tw2, src2, stream); break;
    case 14: e = launch_large_sub_inv<14, SCHED_SHORT_LAST>(work, units, s1, tw2, src2, stream); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if (s1 <= 4) {
    if ((e = stream_grid(batch << s2, &grid)) != hipSuccess) return e;
  } else if ((e = stream_grid(((batch << s2) >> (12 - s1)) * LARGE_THREADS, &grid)) !=
             hipSuccess) {
    return e;
  }
  switch (s1) {
#define HIDFT_TOPI(S1)                                                                          \
  case S1:                                                                                      \
    hipLaunchKernelGGL(large_top_inv_kernel<S1>, dim3(grid), dim3(LARGE_THREADS), 0, stream,    \
                       work, out, ld_out, batch, s2, tw, scale);                                \
    break;
#define HIDFT_TOPI2(S1)                                                                         \
  case S1:                                                                                      \
    hipLaunchKernelGGL(large_top2_inv_kernel<S1>, dim3(grid), dim3(LARGE_THREADS), 0, stream,   \
                       work, out, ld_out, batch, s2, tw, scale);                                \
    break;
    HIDFT_TOPI(1) HIDFT_TOPI(2) HIDFT_TOPI(3) HIDFT_TOPI(4)
    HIDFT_TOPI2(5) HIDFT_TOPI2(6) HIDFT_TOPI2(7) HIDFT_TOPI2(8)
#undef HIDFT_TOPI
#undef HIDFT_TOPI2
    case TOP3_S1: {
      static OccupancyCache cache3;
      unsigned grid3 = 0;
      if ((e = top3_grid((const void*)large_top3_inv_kernel, TOP3_INV_THREADS, TOP3_INV_COLS,
                         cache3, batch, s2, &grid3)) != hipSuccess)
        return e;
      hipLaunchKernelGGL(large_top3_inv_kernel, dim3(grid3), dim3(TOP3_INV_THREADS), 0, stream,
                         work, out, ld_out, batch, s2, tw, scale);
      break;
    }
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free Shift-and-Sample entry point: the shifted
// Hi-DFT outputs of a chunk of signals, [signal][shift][node], instead of a
// caller's workspace.  In host code `scratch` names a host-side stand-in, not
// device memory: every host use goes through the address hipGetSymbolAddress
// returns for the current device, looked up once per device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) float2 scratch[SAS_SCRATCH_BYTES / sizeof(float2)];

constexpr int SCRATCH_MAX_DEVICES = 64;

hipError_t sas_scratch(void** ptr) {
  static std::atomic<void*> per_device[SCRATCH_MAX_DEVICES];
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
  void* p = per_device[dev].load(std::memory_order_acquire);
  if (p == nullptr) {
    // Racing first calls on a device each look up the same address.
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    per_device[dev].store(p, std::memory_order_release);
  }
  *ptr = p;
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Plain per-signal method (baseline): one block per launch, one signal.
//
// Samples are permuted into the recursion order p = bitrev_S(a) in LDS, then
// each radix-2 stage of Lemma 3 runs over the p-order array between two
// barriers: stage u pairs p and p + 2^{u-1} with the twiddle of
// q_lo = p mod 2^{u-1}.  The output for J[t] sits at p = q(J[t]).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t brev_bits(uint32_t x, int nbits) {
  return nbits == 0 ? 0u : (__brev(x) >> (32 - nbits));
}

__global__ void __launch_bounds__(256)
hidft_plain_kernel(const float2* __restrict__ in, float2* __restrict__ out, int S,
                   const float2* __restrict__ tw, const uint16_t* __restrict__ src,
                   float scale) {
  extern __shared__ float2 X[];
  const int k = 1 << S;
  for (int a = threadIdx.x; a < k; a += blockDim.x) X[brev_bits(a, S)] = in[a];
  __syncthreads();
  for (int u = 1; u <= S; ++u) {
    const int h = 1 << (u - 1);
    for (int b = threadIdx.x; b < k / 2; b += blockDim.x) {
      const int q_lo = b & (h - 1);
      const int p = ((b >> (u - 1)) << u) + q_lo;
      const float2 w = tw[(h - 1) + brev_bits(q_lo, u - 1)];
      butterfly(X[p], X[p + h], w);
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < k; t += blockDim.x) {
    const float2 x = X[brev_bits(src[t], S)];
    out[t] = make_float2(x.x * scale, x.y * scale);
  }
}

hipError_t launch_plain(uint32_t s, const float2* in, float2* out, const float2* tw,
                        const uint16_t* src, float scale, hipStream_t stream) {
  if (s == 0) {
    hipLaunchKernelGGL(hidft_k1_kernel, dim3(1), dim3(1), 0, stream, in, 1, out, 1,
                       (uint64_t)1, scale);
    return hipGetLastError();
  }
  const size_t lds = ((size_t)1 << s) * sizeof(float2);
  // The LDS limit is raised on the first call; racing threads set the same value.
  static std::atomic<bool> attr_set{false};
  if (!attr_set.load(std::memory_order_acquire)) {
    hipError_t e = hipFuncSetAttribute((const void*)hidft_plain_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(((size_t)1 << HIDFT_MAX_LOG2_K_DEVICE) * sizeof(float2)));
    if (e != hipSuccess) return e;
    attr_set.store(true, std::memory_order_release);
  }
  int threads = (1 << s) / 2;
  if (threads < 64) threads = 64;
  if (threads > 256) threads = 256;
  hipLaunchKernelGGL(hidft_plain_kernel, dim3(1), dim3(threads), lds, stream, in, out, (int)s,
                     tw, src, scale);
  return hipGetLastError();
}

}  // namespace hidft
