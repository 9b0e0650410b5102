// Element-wise energy convolution of two energy-resolved quantities, the
// form of the scattering terms (Sec. "Energy Convolutions", Eq. interaction):
//     B[k][i] = s * sum_{k'} X1'[k + shift - k'][i] * X2[k'][i],
// X1' = X1 or X1 reversed in energy, terms outside [0, n1) left out.  Data
// are energy-major, [energy][element] (the layout of the solver's outputs).
//
// Long sequences: one thread per element, so that every energy row is read
// coalesced, and kConvT consecutive outputs k per thread.  For one k' those outputs need
// kConvT consecutive samples of X1', a window that moves down by one sample
// per k': it is kept in registers as a ring whose slot indices are fixed by
// unrolling kConvT steps, so a step reads one sample of X1' and one of X2
// and does kConvT complex multiply-adds (FP64 vector arithmetic: the work
// is a sum of element-wise products, not a matrix contraction).
#include "qtx_internal.h"

namespace qtx {
namespace {

constexpr int kConvT = 16;          // outputs per thread
constexpr int kConvThreads = 256;   // elements per workgroup

__global__ __launch_bounds__(kConvThreads)
void energy_conv_kernel(const double2* __restrict__ X1, int n1, int rev,
                        const double2* __restrict__ X2, int n2, double2* __restrict__ B,
                        int n_out, int shift, double2 s, long long n_elem, int tiles_k) {
  // The k tiles of one group of elements read the same samples: consecutive
  // work items go to one XCD (consecutive block ids go round robin over the
  // eight XCDs), so those reads share its L2.
  const long long nb = (long long)gridDim.x;
  const long long L = blockIdx.x;
  const long long full = nb / 8 * 8;
  const long long w = L < full ? (L % 8) * (nb / 8) + L / 8 : L;
  const long long g = w / tiles_k;
  const int k0 = (int)(w % tiles_k) * kConvT;
  const long long i = g * kConvThreads + threadIdx.x;
  if (i >= n_elem) return;

  // sample j of X1' at this element (zero outside [0, n1))
  auto x1 = [&](int j) {
    const bool in = j >= 0 && j < n1;
    const int jj = in ? (rev ? n1 - 1 - j : j) : 0;
    double2 v = X1[(long long)jj * n_elem + i];
    if (!in) v = make_double2(0.0, 0.0);
    return v;
  };

  double2 acc[kConvT];
#pragma unroll
  for (int u = 0; u < kConvT; ++u) acc[u] = make_double2(0.0, 0.0);
  // the k' with a term for some output of the tile
  const int lo = max(0, k0 + shift - n1 + 1);
  const int hi = min(n2 - 1, k0 + shift + kConvT - 1);
  if (lo <= hi) {
    // ring: at step q (k' = lo + r0 + q) logical window entry u, the sample
    // X1'(k0 + shift - k' + u), sits in slot (u - q) mod kConvT
    double2 ring[kConvT];
#pragma unroll
    for (int u = 0; u < kConvT; ++u) ring[u] = x1(k0 + shift - lo + u);
    const int count = hi - lo + 1;
    for (int r0 = 0; r0 < count; r0 += kConvT) {
#pragma unroll
      for (int q = 0; q < kConvT; ++q) {
        if (r0 + q < count) {                      // uniform across the workgroup
          const int kp = lo + r0 + q;
          const double2 b = X2[(long long)kp * n_elem + i];
#pragma unroll
          for (int u = 0; u < kConvT; ++u) {
            const double2 a = ring[(u - q + kConvT) % kConvT];
            acc[u].x = fma(a.x, b.x, fma(-a.y, b.y, acc[u].x));
            acc[u].y = fma(a.x, b.y, fma(a.y, b.x, acc[u].y));
          }
          // the entry that leaves the window takes the one that enters
          ring[(kConvT - 1 - q + kConvT) % kConvT] = x1(k0 + shift - kp - 1);
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < kConvT; ++u) {
    const int k = k0 + u;
    if (k < n_out)
      B[(long long)k * n_elem + i] =
          make_double2(s.x * acc[u].x - s.y * acc[u].y, s.x * acc[u].y + s.y * acc[u].x);
  }
}

// Short sequences (n1 + n2 <= kLdsSamples): a workgroup stages the whole
// X1' and X2 sequences of kLdsE consecutive entries in LDS once (X1 stored
// reversed when asked, so that it is X1'), and all output tiles of those
// entries are computed from there, so every input is read from HBM once
// (the kernel above re-reads an entry's inputs for each of its output
// tiles).  Thread (slot, e): entry e, outputs k0 .. k0 + kLdsT - 1 with
// k0 = kLdsT slot + 16 kLdsT m; the same register ring and the same order of
// the sums as above.  8 entries x 400 samples take 50 KB, so three
// workgroups share a CU.
constexpr int kLdsT = 8;                 // outputs per thread
constexpr int kLdsE = 8;                 // entries per workgroup
constexpr int kLdsThreads = kLdsE * 16;  // 16 output tiles per pass
constexpr int kLdsSamples = 400;         // largest n1 + n2

__global__ __launch_bounds__(kLdsThreads)
void energy_conv_lds_kernel(const double2* __restrict__ X1, int n1, int rev,
                            const double2* __restrict__ X2, int n2, double2* __restrict__ B,
                            int n_out, int shift, double2 s, long long n_elem) {
  __shared__ double2 S[kLdsSamples * kLdsE];   // [sample][entry]: X1' then X2
  const long long i0 = (long long)blockIdx.x * kLdsE;
  const int t = threadIdx.x;
  const int ns = n1 + n2;
  // consecutive threads take consecutive entries of one sample row; a
  // compile-time trip count keeps all of a thread's loads in flight at once
  constexpr int kPer = (kLdsSamples * kLdsE + kLdsThreads - 1) / kLdsThreads;
  double2 v[kPer];
#pragma unroll
  for (int m = 0; m < kPer; ++m) {
    const int idx = t + m * kLdsThreads;
    const int sr = idx / kLdsE, e = idx % kLdsE;
    const long long i = i0 + e;
    v[m] = make_double2(0.0, 0.0);
    if (idx < ns * kLdsE && i < n_elem)
      v[m] = sr < n1 ? X1[(long long)(rev ? n1 - 1 - sr : sr) * n_elem + i]
                     : X2[(long long)(sr - n1) * n_elem + i];
  }
#pragma unroll
  for (int m = 0; m < kPer; ++m) {
    const int idx = t + m * kLdsThreads;
    if (idx < ns * kLdsE) S[idx] = v[m];
  }
  __syncthreads();
  const int e = t % kLdsE, slot = t / kLdsE;
  const long long i = i0 + e;
  const double2* S2 = S + n1 * kLdsE;
  // sample j of X1' at this entry (zero outside [0, n1))
  auto x1 = [&](int j) {
    const bool in = j >= 0 && j < n1;
    double2 v = S[(in ? j : 0) * kLdsE + e];
    if (!in) v = make_double2(0.0, 0.0);
    return v;
  };
  for (int k0 = slot * kLdsT; k0 < n_out; k0 += 16 * kLdsT) {
    double2 acc[kLdsT];
#pragma unroll
    for (int u = 0; u < kLdsT; ++u) acc[u] = make_double2(0.0, 0.0);
    const int lo = max(0, k0 + shift - n1 + 1);
    const int hi = min(n2 - 1, k0 + shift + kLdsT - 1);
    if (lo <= hi) {
      double2 ring[kLdsT];
#pragma unroll
      for (int u = 0; u < kLdsT; ++u) ring[u] = x1(k0 + shift - lo + u);
      const int count = hi - lo + 1;
      const int full = count / kLdsT * kLdsT;
      // whole blocks of kLdsT steps: no guards, so all of a block's LDS
      // reads are issued ahead of its multiply-adds
      for (int r0 = 0; r0 < full; r0 += kLdsT) {
        double2 bq[kLdsT], xq[kLdsT];
#pragma unroll
        for (int q = 0; q < kLdsT; ++q) {
          const int kp = lo + r0 + q;
          bq[q] = S2[kp * kLdsE + e];
          xq[q] = x1(k0 + shift - kp - 1);
        }
#pragma unroll
        for (int q = 0; q < kLdsT; ++q) {
#pragma unroll
          for (int u = 0; u < kLdsT; ++u) {
            const double2 a = ring[(u - q + kLdsT) % kLdsT];
            acc[u].x = fma(a.x, bq[q].x, fma(-a.y, bq[q].y, acc[u].x));
            acc[u].y = fma(a.x, bq[q].y, fma(a.y, bq[q].x, acc[u].y));
          }
          ring[(kLdsT - 1 - q + kLdsT) % kLdsT] = xq[q];
        }
      }
      // the last, partial block
#pragma unroll
      for (int q = 0; q < kLdsT; ++q) {
        if (full + q < count) {
          const int kp = lo + full + q;
          const double2 b = S2[kp * kLdsE + e];
#pragma unroll
          for (int u = 0; u < kLdsT; ++u) {
            const double2 a = ring[(u - q + kLdsT) % kLdsT];
            acc[u].x = fma(a.x, b.x, fma(-a.y, b.y, acc[u].x));
            acc[u].y = fma(a.x, b.y, fma(a.y, b.x, acc[u].y));
          }
          ring[(kLdsT - 1 - q + kLdsT) % kLdsT] = x1(k0 + shift - kp - 1);
        }
      }
    }
    if (i < n_elem) {
#pragma unroll
      for (int u = 0; u < kLdsT; ++u) {
        const int k = k0 + u;
        if (k < n_out)
          B[(long long)k * n_elem + i] =
              make_double2(s.x * acc[u].x - s.y * acc[u].y, s.x * acc[u].y + s.y * acc[u].x);
      }
    }
  }
}

}  // namespace

hipError_t launch_energy_convolution(const void* X1, int n1, int rev, const void* X2, int n2,
                                     void* B, int n_out, int shift, double s_re, double s_im,
                                     long long n_elem, hipStream_t st) {
  if (n_elem <= 0 || n_out <= 0) return hipSuccess;
  if (n1 + n2 <= kLdsSamples) {
    const long long nb = (n_elem + kLdsE - 1) / kLdsE;
    if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(energy_conv_lds_kernel, dim3((unsigned)nb), dim3(kLdsThreads), 0, st,
                       (const double2*)X1, n1, rev, (const double2*)X2, n2, (double2*)B, n_out,
                       shift, make_double2(s_re, s_im), n_elem);
    return hipGetLastError();
  }
  const long long groups = (n_elem + kConvThreads - 1) / kConvThreads;
  const int tiles_k = (n_out + kConvT - 1) / kConvT;
  const long long nb = groups * tiles_k;
  if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(energy_conv_kernel, dim3((unsigned)nb), dim3(kConvThreads), 0, st,
                     (const double2*)X1, n1, rev, (const double2*)X2, n2, (double2*)B, n_out,
                     shift, make_double2(s_re, s_im), n_elem, tiles_k);
  return hipGetLastError();
}

}  // namespace qtx
