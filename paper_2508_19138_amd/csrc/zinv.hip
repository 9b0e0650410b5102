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
// Blocking: the columns are processed in panels of kPanel.  One workgroup
// per matrix factors the panel (rows held in registers, one row per thread
// and pass), producing the eliminated panel columns in place.  The effect on
// every other column j is then the rank-kPanel update
//     A[:, j] += Panel''[:, :] * A[pivot rows, j]
// where Panel'' equals the eliminated panel except that 1 is subtracted at
// each (pivot row, its column).  That update is one complex GEMM on the
// matrix cores (beta = 1, in place).  The gathered pivot rows have their
// panel columns set to zero, so the panel columns pass through unchanged.
#include "qtx_internal.h"

namespace qtx {
namespace {

constexpr int kInvThreads = 256;

template <int R>
__global__ __launch_bounds__(kInvThreads)
void gj_panel_kernel(double2* __restrict__ S, long long sS, int b, int k0,
                     double2* __restrict__ panel, double2* __restrict__ brow,
                     int* __restrict__ perm, int* __restrict__ used,
                     int* __restrict__ info, int code_base) {
  constexpr int NB = kPanel;
  __shared__ double redv[kInvThreads / 64];
  __shared__ int redr[kInvThreads / 64];
  __shared__ int redbad[kInvThreads / 64];
  __shared__ double2 prow[NB];
  __shared__ int pivs[NB];

  const int e = blockIdx.x;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  double2* A = S + e * sS;
  int* pe = perm + (long long)e * b;
  int* ue = used + (long long)e * b;
  double2* pan = panel + (long long)e * b * NB;
  double2* br = brow + (long long)e * NB * b;
  const int nbe = min(NB, b - k0);

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

  int first_bad = 0;   // set by thread 0 only
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
    // bi is a valid unused row whenever b - k0 - c > 0 rows remain unused.
    const int p = (bi == 0x7fffffff) ? 0 : bi;
    if (t == 0 && first_bad == 0) {
      const int code = code_base > 0 ? code_base : 1 + k0 + c;
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
    if (info && first_bad != 0 && info[e] == 0) info[e] = first_bad;
  }
  // gathered pivot rows of the original matrix (panel columns zeroed)
  for (int c = 0; c < NB; ++c) {
    const int p = (c < nbe) ? pivs[c] : -1;
    for (int j = t; j < b; j += kInvThreads) {
      double2 v = make_double2(0.0, 0.0);
      if (p >= 0 && (j < k0 || j >= k0 + nbe)) v = A[(long long)p * b + j];
      br[(long long)c * b + j] = v;
    }
  }
}

// X[k][c] = Y[p_k][pinv(c)] with pinv(p_j) = j.
__global__ __launch_bounds__(256)
void gj_permute_kernel(const double2* __restrict__ Y, long long sY,
                       double2* __restrict__ X, long long sX, int b,
                       const int* __restrict__ perm, int rows_per_block) {
  extern __shared__ int sh[];
  int* pinv = sh;
  int* pk = sh + b;
  const int e = blockIdx.y;
  const int* pe = perm + (long long)e * b;
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
  const double2* Ye = Y + e * sY;
  double2* Xe = X + e * sX;
  const int r0 = blockIdx.x * rows_per_block;
  const int r1 = min(b, r0 + rows_per_block);
  for (int k = r0; k < r1; ++k) {
    const long long src = (long long)pk[k] * b;
    for (int c = threadIdx.x; c < b; c += blockDim.x)
      Xe[(long long)k * b + c] = Ye[src + pinv[c]];
  }
}

template <int R>
hipError_t launch_panel(int b, void* S, long long sS, int k0, int batch,
                        const InvWork& w, int* info, int code_base,
                        hipStream_t s) {
  hipLaunchKernelGGL(gj_panel_kernel<R>, dim3(batch), dim3(kInvThreads), 0, s,
                     (double2*)S, sS, b, k0, (double2*)w.panel,
                     (double2*)w.brow, w.perm, w.used, info, code_base);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_zinv(int b, void* S, long long sS, void* X, long long sX,
                       int batch, const InvWork& w, int* info, int code_base,
                       hipStream_t s) {
  if (batch <= 0 || b <= 0) return hipSuccess;
  const int R = (b + kInvThreads - 1) / kInvThreads;
  if (R > 4) return hipErrorInvalidValue;     // b <= 1024
  for (int k0 = 0; k0 < b; k0 += kPanel) {
    hipError_t err;
    switch (R) {
      case 1: err = launch_panel<1>(b, S, sS, k0, batch, w, info, code_base, s); break;
      case 2: err = launch_panel<2>(b, S, sS, k0, batch, w, info, code_base, s); break;
      case 3: err = launch_panel<3>(b, S, sS, k0, batch, w, info, code_base, s); break;
      default: err = launch_panel<4>(b, S, sS, k0, batch, w, info, code_base, s); break;
    }
    if (err != hipSuccess) return err;
    if (b > kPanel) {
      GemmArgs g{};
      g.M = b; g.N = b; g.K = kPanel;
      g.lda = kPanel; g.ldb = b; g.ldc = b; g.ldd = b;
      g.batch = batch; g.ngroups = 1;
      g.g[0].A = w.panel; g.g[0].sA = (long long)b * kPanel;
      g.g[0].B = w.brow;  g.g[0].sB = (long long)kPanel * b;
      g.g[0].C = S;       g.g[0].sC = sS;
      g.g[0].D = S;       g.g[0].sD = sS;
      g.g[0].alpha = zc{1.0, 0.0};
      g.g[0].beta = zc{1.0, 0.0};
      err = launch_zgemm('N', 'N', g, s);
      if (err != hipSuccess) return err;
    }
  }
  const int rpb = 8;
  dim3 grid((b + rpb - 1) / rpb, batch);
  hipLaunchKernelGGL(gj_permute_kernel, grid, dim3(256), 2 * b * sizeof(int), s,
                     (const double2*)S, sS, (double2*)X, sX, b, w.perm, rpb);
  return hipGetLastError();
}

}  // namespace qtx
