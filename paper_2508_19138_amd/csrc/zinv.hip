// Batched inverse of complex128 b x b blocks: blocked Gauss-Jordan
// elimination with partial pivoting (largest |z|^2 in the pivot column,
// ties to the lowest row index).
//
// Rows are never swapped.  Pivoting is implicit: column k is eliminated with
// the pivot row p_k chosen among the rows not used yet, and row p_k plays
// the role of row k.  After all columns the in-place result Y satisfies
//     Y[p_k][j] = (P A)^{-1}[k][j],  P A = rows of A in the order p_0, p_1, ...
// and A^{-1} = (P A)^{-1} P, i.e.  A^{-1}[k][p_j] = Y[p_k][j]; the final
// kernel applies that permutation while copying into the destination.
//
// Blocking, two levels.  Eliminating a set K of columns with pivot rows pK
// changes every other column j by the rank-|K| update
//     A[:, j] += Panel''[:, K] * A[pK, j]
// where Panel'' is the eliminated block of columns minus the identity at the
// (pivot row, column) positions; this holds however the columns of K were
// eliminated.  So the columns are taken in super-panels of kSuper, each made
// of panels of kPanel.  One workgroup per matrix factors a panel (rows held
// in registers, one row per thread and pass) and gathers its pivot rows
// restricted to the super-panel; a rank-kPanel product updates the rest of
// the super-panel only.  After the last panel, the eliminated super-panel
// and its pivot rows outside it are gathered and one rank-kSuper product on
// the matrix cores updates the whole matrix.  Gathered pivot rows carry
// zeros in the columns being eliminated, so those pass through unchanged.
#include "qtx_internal.h"

namespace qtx {
namespace {

template <int R>
__global__ __launch_bounds__(kInvThreads)
void gj_panel_kernel(FlatLaunch L, int k0) {
  constexpr int NB = kPanel;
  __shared__ double redv[kInvThreads / 64];
  __shared__ int redr[kInvThreads / 64];
  __shared__ int redbad[kInvThreads / 64];
  __shared__ double2 prow[NB];
  __shared__ int pivs[NB];

  const int di = find_desc(L.prefix, L.nd, blockIdx.x);
  const InvDesc& d = ((const InvDesc*)L.desc)[di];
  const int e = blockIdx.x - L.prefix[di];
  const int b = d.b;
  if (k0 >= b) return;                       // this matrix has no such panel
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  double2* A = (double2*)d.S + e * d.sS;
  int* pe = d.perm + (long long)e * b;
  int* ue = d.used + (long long)e * b;
  double2* pan = (double2*)d.panel + (long long)e * b * NB;
  double2* br = (double2*)d.brow + (long long)e * NB * b;
  const int nbe = min(NB, b - k0);
  const int lo = k0 - k0 % kSuper;                // current super-panel
  const int hi = min(b, lo + kSuper);

  double2 a[R][NB];
  int u[R];      // row already used as a pivot
  int pc[R];     // panel column this row pivots (-1 if none)
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int r = t + q * kInvThreads;
    pc[q] = -1;
    u[q] = 1;
    if (r < b) {
      u[q] = (k0 == 0) ? 0 : ue[r];
#pragma unroll
      for (int c = 0; c < NB; ++c)
        a[q][c] = (c < nbe) ? A[(long long)r * b + k0 + c] : make_double2(0.0, 0.0);
    } else {
#pragma unroll
      for (int c = 0; c < NB; ++c) a[q][c] = make_double2(0.0, 0.0);
    }
  }

  int first_bad = 0;   // meaningful in thread 0 only
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    if (c >= nbe) continue;      // uniform across the workgroup
    // ---- pivot search over unused rows -------------------------------
    double bv = -1.0;
    int bi = 0x7fffffff;
    int bad = 0;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int r = t + q * kInvThreads;
      if (r < b && !u[q]) {
        const double v = a[q][c].x * a[q][c].x + a[q][c].y * a[q][c].y;
        if (!(v <= 1.7976931348623157e308)) bad = 1;     // NaN or Inf
        else if (v > bv) { bv = v; bi = r; }
      }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const double ov = __shfl_xor(bv, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      const int ob = __shfl_xor(bad, off, 64);
      if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
      bad |= ob;
    }
    if (lane == 0) { redv[wave] = bv; redr[wave] = bi; redbad[wave] = bad; }
    __syncthreads();
    bv = redv[0]; bi = redr[0]; bad = redbad[0];
#pragma unroll
    for (int w = 1; w < kInvThreads / 64; ++w) {
      const double ov = redv[w];
      const int oi = redr[w];
      if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
      bad |= redbad[w];
    }
    // An unused row always remains (b - k0 - c > 0), so bi is a valid row
    // unless every candidate was non-finite; then row 0 keeps indices in
    // range and the failure is reported through info.
    const int p = (bi == 0x7fffffff) ? 0 : bi;
    if (t == 0 && first_bad == 0) {
      const int code = d.code > 0 ? d.code : 1 + k0 + c;
      if (bad) first_bad = -code;
      else if (bv <= 0.0) first_bad = code;
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int r = t + q * kInvThreads;
      if (r == p) {
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) prow[cc] = a[q][cc];
        u[q] = 1;
        pc[q] = c;
      }
    }
    if (t == 0) pivs[c] = p;
    __syncthreads();
    // ---- eliminate column k0 + c from every row ---------------------
    const double2 inv = crecip(prow[c]);
    double2 ps[NB];
#pragma unroll
    for (int cc = 0; cc < NB; ++cc) ps[cc] = (cc == c) ? inv : cmul(prow[cc], inv);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int r = t + q * kInvThreads;
      if (r >= b) continue;
      if (r == p) {
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) a[q][cc] = ps[cc];
      } else {
        const double2 f = a[q][c];
        a[q][c] = make_double2(0.0, 0.0);
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) a[q][cc] = csub(a[q][cc], cmul(f, ps[cc]));
      }
    }
  }

  // ---- write back the panel, Panel'' and the gathered pivot rows ---------
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int r = t + q * kInvThreads;
    if (r >= b) continue;
    ue[r] = u[q];
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      if (c < nbe) A[(long long)r * b + k0 + c] = a[q][c];
      double2 v = a[q][c];
      if (pc[q] == c) v.x -= 1.0;
      pan[(long long)r * NB + c] = v;
    }
  }
  if (t == 0) {
    for (int c = 0; c < nbe; ++c) pe[k0 + c] = pivs[c];
    if (d.info) {
      int* inf = d.info + e;
      const int cur = (k0 == 0 && d.reset_info) ? 0 : *inf;
      if (cur == 0) *inf = first_bad;
    }
  }
  // pivot rows within the super-panel (this panel's columns zeroed)
  for (int c = 0; c < NB; ++c) {
    const int p = (c < nbe) ? pivs[c] : -1;
    for (int j = lo + t; j < hi; j += kInvThreads) {
      double2 v = make_double2(0.0, 0.0);
      if (p >= 0 && (j < k0 || j >= k0 + nbe)) v = A[(long long)p * b + j];
      br[(long long)c * b + j] = v;
    }
  }
}

// spanel[r][c] = A[r][K0 + c] - (r == p_{K0+c}),  sbrow[c][j] = A[p_{K0+c}][j]
// outside [K0, K0 + kSuper) and 0 inside; c beyond the matrix are zero.
__global__ __launch_bounds__(256)
void gj_super_gather_kernel(FlatLaunch L, int K0) {
  const int di = find_desc(L.prefix, L.nd, blockIdx.x);
  const InvDesc& d = ((const InvDesc*)L.desc)[di];
  const int b = d.b;
  const int chunks = super_gather_chunks(b);
  const int local = blockIdx.x - L.prefix[di];
  const long long e = local / chunks;
  const long long q0 = (long long)(local % chunks) * kGatherItems;
  const double2* A = (const double2*)d.S + e * d.sS;
  const int* pe = d.perm + e * b;
  double2* sp = (double2*)d.spanel + e * (long long)b * kSuper;
  double2* sb = (double2*)d.sbrow + e * (long long)kSuper * b;
  const int spe = min(kSuper, b - K0);
  const long long half = (long long)b * kSuper;
  const long long q1 = min(q0 + kGatherItems, 2 * half);
  for (long long q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
    if (q < half) {
      const int r = (int)(q / kSuper), c = (int)(q % kSuper);
      double2 v = make_double2(0.0, 0.0);
      if (c < spe) {
        v = A[(long long)r * b + K0 + c];
        if (pe[K0 + c] == r) v.x -= 1.0;
      }
      sp[q] = v;
    } else {
      const long long qq = q - half;
      const int c = (int)(qq / b), j = (int)(qq % b);
      double2 v = make_double2(0.0, 0.0);
      if (c < spe && (j < K0 || j >= K0 + spe)) {
        const int p = pe[K0 + c];
        if (p >= 0 && p < b) v = A[(long long)p * b + j];
      }
      sb[qq] = v;
    }
  }
}

// X[k][c] = Y[p_k][pinv(c)] with pinv(p_j) = j; kPermRows rows per workgroup.
__global__ __launch_bounds__(256)
void gj_permute_kernel(FlatLaunch L) {
  __shared__ int pinv[1024];
  __shared__ int pk[1024];
  const int di = find_desc(L.prefix, L.nd, blockIdx.x);
  const InvDesc& d = ((const InvDesc*)L.desc)[di];
  const int b = d.b;
  const int chunks = (b + kPermRows - 1) / kPermRows;
  const int local = blockIdx.x - L.prefix[di];
  const int e = local / chunks;
  const int r0 = (local % chunks) * kPermRows;
  const int* pe = d.perm + (long long)e * b;
  // Pivots are distinct rows unless a non-finite column was met (flagged
  // through info); starting from the identity keeps every index in range.
  for (int j = threadIdx.x; j < b; j += blockDim.x) {
    pinv[j] = j;
    const int pj = pe[j];
    pk[j] = (pj >= 0 && pj < b) ? pj : j;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < b; j += blockDim.x) pinv[pk[j]] = j;
  __syncthreads();
  const double2* Ye = (const double2*)d.S + e * d.sS;
  double2* Xe = (double2*)d.X + e * d.sX;
  const int r1 = min(b, r0 + kPermRows);
  for (int k = r0; k < r1; ++k) {
    const long long src = (long long)pk[k] * b;
    for (int c = threadIdx.x; c < b; c += blockDim.x)
      Xe[(long long)k * b + c] = Ye[src + pinv[c]];
  }
}

}  // namespace

hipError_t launch_inv_panel(int R, int k0, const FlatLaunch& l, hipStream_t s) {
  if (l.total <= 0) return hipSuccess;
  switch (R) {
    case 1: hipLaunchKernelGGL(gj_panel_kernel<1>, dim3(l.total), dim3(kInvThreads), 0, s, l, k0); break;
    case 2: hipLaunchKernelGGL(gj_panel_kernel<2>, dim3(l.total), dim3(kInvThreads), 0, s, l, k0); break;
    case 3: hipLaunchKernelGGL(gj_panel_kernel<3>, dim3(l.total), dim3(kInvThreads), 0, s, l, k0); break;
    case 4: hipLaunchKernelGGL(gj_panel_kernel<4>, dim3(l.total), dim3(kInvThreads), 0, s, l, k0); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_inv_super_gather(int K0, const FlatLaunch& l, hipStream_t s) {
  if (l.total <= 0) return hipSuccess;
  hipLaunchKernelGGL(gj_super_gather_kernel, dim3(l.total), dim3(256), 0, s, l, K0);
  return hipGetLastError();
}

hipError_t launch_inv_permute(const FlatLaunch& l, hipStream_t s) {
  if (l.total <= 0) return hipSuccess;
  hipLaunchKernelGGL(gj_permute_kernel, dim3(l.total), dim3(256), 0, s, l);
  return hipGetLastError();
}

}  // namespace qtx
