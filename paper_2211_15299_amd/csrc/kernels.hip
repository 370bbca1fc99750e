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

// LDS padding: one spare slot after every 16 complex values keeps the strided
// accesses of the radix-16 groups spread over the 64 LDS banks.
__device__ __forceinline__ int lds_pad(int a) { return a + (a >> 4); }

template <int S>
struct FusedShape {
  static constexpr int RHO = S < 4 ? S : 4;                      // log2 points per thread
  static constexpr int R = 1 << RHO;
  static constexpr int K = 1 << S;
  static constexpr int T = K / R;                                // threads per signal
  static constexpr int SPB = T >= 256 ? 1 : 256 / T;             // signals per block
  static constexpr int THREADS = T * SPB;
  static constexpr int G = S == 0 ? 0 : (S + RHO - 1) / RHO;     // radix groups
  static constexpr int G1 = S == 0 ? 0 : S - (G - 1) * RHO;      // stages in group 1
  static constexpr int PADK = K + (K >> 4);                      // LDS slots per signal
  static constexpr size_t LDS_BYTES = (size_t)SPB * PADK * sizeof(float2);
};

// ---------------------------------------------------------------------------
// Fused batched transform: one signal per T threads, SPB signals per block.
//
// Group 1 (stages 1..G1, the top G1 bits of a) runs straight from the global
// load: thread tau holds a = tau + c*T for c < R, so each load instruction of
// a wavefront reads 64 consecutive samples.  Every later group takes RHO = 4
// stages (radix 16) on the next lower four bits, through LDS.  After the last
// group the block gathers the outputs in the caller's order of J, scales by
// N/k and stores them coalesced.
// ---------------------------------------------------------------------------
template <int S>
__global__ void __launch_bounds__(FusedShape<S>::THREADS)
hidft_fused_kernel(const float2* __restrict__ in, int64_t ld_in, float2* __restrict__ out,
                   int64_t ld_out, uint64_t batch, const float2* __restrict__ tw,
                   const uint16_t* __restrict__ src, float scale) {
  using Sh = FusedShape<S>;
  constexpr int RHO = Sh::RHO, R = Sh::R, T = Sh::T, SPB = Sh::SPB, G = Sh::G, G1 = Sh::G1;
  extern __shared__ float2 lds[];

  const int tid = threadIdx.x;
  const int slot = tid / T;
  const int tau = tid - slot * T;
  const uint64_t sig = (uint64_t)blockIdx.x * SPB + slot;
  const bool valid = sig < batch;
  float2* L = lds + slot * Sh::PADK;

  float2 v[R];
  {
    const float2* row = in + (valid ? sig : 0) * (uint64_t)ld_in;
#pragma unroll
    for (int c = 0; c < R; ++c) v[c] = valid ? row[c * T + tau] : make_float2(0.f, 0.f);
  }

  // Group 1: stage u pairs bit RHO-u of c; the twiddle index is the top u-1
  // bits of c, the same for every thread (scalar loads).
#pragma unroll
  for (int u = 1; u <= G1; ++u) {
    const int bit = RHO - u;
#pragma unroll
    for (int c = 0; c < R; ++c) {
      if (c & (1 << bit)) continue;
      const float2 w = tw[(1 << (u - 1)) - 1 + (c >> (bit + 1))];
      butterfly(v[c], v[c | (1 << bit)], w);
    }
  }
#pragma unroll
  for (int c = 0; c < R; ++c) L[lds_pad(c * T + tau)] = v[c];

  // Groups 2..G: bits [lo, lo + RHO) with lo = S - G1 - (g-1)*RHO.  Each
  // thread reads and writes back the same 16 slots, so one barrier per group
  // suffices.
#pragma unroll
  for (int g = 2; g <= G; ++g) {
    const int lo = S - G1 - (g - 1) * RHO;
    const int a_lo = tau & ((1 << lo) - 1);
    const int a_hi = tau >> lo;
    const int base = a_lo + (a_hi << (lo + RHO));
    __syncthreads();
#pragma unroll
    for (int c = 0; c < R; ++c) v[c] = L[lds_pad(base + (c << lo))];
#pragma unroll
    for (int t = 0; t < RHO; ++t) {
      const int u = S - lo - RHO + 1 + t;
      const int bit = RHO - 1 - t;
      const float2* twu = tw + ((1 << (u - 1)) - 1) + (a_hi << t);
#pragma unroll
      for (int c = 0; c < R; ++c) {
        if (c & (1 << bit)) continue;
        const float2 w = twu[c >> (RHO - t)];
        butterfly(v[c], v[c | (1 << bit)], w);
      }
    }
#pragma unroll
    for (int c = 0; c < R; ++c) L[lds_pad(base + (c << lo))] = v[c];
  }
  __syncthreads();

  if (valid) {
    float2* orow = out + sig * (uint64_t)ld_out;
#pragma unroll
    for (int c = 0; c < R; ++c) {
      const int t = c * T + tau;
      const float2 x = L[lds_pad((int)src[t])];
      orow[t] = make_float2(x.x * scale, x.y * scale);
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

template <int S>
static hipError_t launch_fused_s(const float2* in, int64_t ld_in, float2* out, int64_t ld_out,
                                 uint64_t batch, const float2* tw, const uint16_t* src,
                                 float scale, hipStream_t stream) {
  using Sh = FusedShape<S>;
  static bool attr_set = false;  // benign race: every thread sets the same value
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)hidft_fused_kernel<S>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)Sh::LDS_BYTES);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const uint64_t blocks = (batch + Sh::SPB - 1) / Sh::SPB;
  if (blocks > 0x7fffffffULL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(hidft_fused_kernel<S>, dim3((unsigned)blocks), dim3(Sh::THREADS),
                     Sh::LDS_BYTES, stream, in, ld_in, out, ld_out, batch, tw, src, scale);
  return hipGetLastError();
}

hipError_t launch_fused(uint32_t s, const float2* in, int64_t ld_in, float2* out,
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
    return launch_fused_s<S>(in, ld_in, out, ld_out, batch, tw, src, scale, stream);
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
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)hidft_plain_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(((size_t)1 << HIDFT_MAX_LOG2_K_DEVICE) * sizeof(float2)));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  int threads = (1 << s) / 2;
  if (threads < 64) threads = 64;
  if (threads > 256) threads = 256;
  hipLaunchKernelGGL(hidft_plain_kernel, dim3(1), dim3(threads), lds, stream, in, out, (int)s,
                     tw, src, scale);
  return hipGetLastError();
}

}  // namespace hidft
