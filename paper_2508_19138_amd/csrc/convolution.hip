// Element-wise energy convolution of two energy-resolved quantities, the
// form of the scattering terms (Sec. "Energy Convolutions", Eq. interaction):
//     B[k][i] = s * sum_{k'} X1'[k + shift - k'][i] * X2[k'][i],
// X1' = X1 or X1 reversed in energy, terms outside [0, n1) left out.  Data
// are energy-major, [energy][element] (the layout of the solver's outputs).
//
// One thread per element, so that every energy row is read coalesced, and
// kConvT consecutive outputs k per thread.  For one k' those outputs need
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

}  // namespace

hipError_t launch_energy_convolution(const void* X1, int n1, int rev, const void* X2, int n2,
                                     void* B, int n_out, int shift, double s_re, double s_im,
                                     long long n_elem, hipStream_t st) {
  if (n_elem <= 0 || n_out <= 0) return hipSuccess;
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
