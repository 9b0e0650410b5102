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

// Pivot search key of a candidate row r with |z|^2 = v (finite, >= 0): the
// bits of v with the low 10 mantissa bits replaced by 1023 - r.  Keys order
// as v (to 42 mantissa bits) and then by lowest row, so the maximum key is
// the partial-pivoting choice and names its row; non-candidates use -1.
__device__ __forceinline__ double pivot_key(double v, int r) {
  const unsigned long long u = ((unsigned long long)__double_as_longlong(v) & ~1023ull) |
                               (unsigned long long)(1023 - r);
  return __longlong_as_double((long long)u);
}
__device__ __forceinline__ int pivot_row(double key) {
  return 1023 - (int)((unsigned long long)__double_as_longlong(key) & 1023ull);
}

// x moved across lanes by a DPP pattern (both 32-bit halves)
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(v & 0xffffffff), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Maximum over the 64 lanes of a wave, returned in every lane: within rows
// of 16 lanes by DPP (quad xor 1, quad xor 2, half-row mirror, row mirror,
// after which every lane holds its row's maximum), then across the four
// rows through scalar reads of one lane per row.
__device__ __forceinline__ double lane_read(double x, int l) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffff), l);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double wave_max(double x) {
  x = fmax(x, dpp_move<0xB1>(x));     // quad_perm [1,0,3,2]
  x = fmax(x, dpp_move<0x4E>(x));     // quad_perm [2,3,0,1]
  x = fmax(x, dpp_move<0x141>(x));    // row_half_mirror
  x = fmax(x, dpp_move<0x140>(x));    // row_mirror
  return fmax(fmax(lane_read(x, 0), lane_read(x, 16)), fmax(lane_read(x, 32), lane_read(x, 48)));
}

// One division: z is scaled by an exact power of two so that |z'|^2 lies in
// [1, 8), then 1/z = conj(z') / |z'|^2 scaled back.
__device__ __forceinline__ double2 crecip_scaled(double2 z) {
  const double s = fmax(fabs(z.x), fabs(z.y));
  if (s == 0.0) return make_double2(1.0 / s, 0.0);   // inf: caller flags it
  int ex;
  (void)frexp(s, &ex);
  const double xr = ldexp(z.x, -ex), xi = ldexp(z.y, -ex);
  const double r = 1.0 / (xr * xr + xi * xi);
  return make_double2(ldexp(xr * r, -ex), ldexp(-xi * r, -ex));
}

template <int R>
__global__ __launch_bounds__(kInvThreads)
void gj_panel_kernel(FlatLaunch L, int k0) {
  constexpr int NB = kPanel;
  constexpr int NW = kInvThreads / 64;
  // per column: each wave publishes its best key and that candidate's row;
  // double buffered by column parity so one barrier per column suffices
  __shared__ double keyS[2][NW];
  __shared__ int badS[2][NW];
  __shared__ double2 rowS[2][NW][NB];
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
  const int code0 = d.code;

  // Panel rows move between HBM and registers through LDS: 16 lanes per
  // row in HBM (256-byte segments), one row per thread in registers.
  __shared__ double2 stage[kInvThreads][NB + 1];
  __shared__ int pcS[kInvThreads];
  double2 a[R][NB];
  int u[R];      // row already used as a pivot
  int pc[R];     // panel column this row pivots (-1 if none)
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int r0 = q * kInvThreads;
    const int r = r0 + t;
    pc[q] = -1;
    u[q] = 1;
    if (r < b) u[q] = (k0 == 0) ? 0 : ue[r];
    if (r0 < b) {                           // uniform across the workgroup
      // unconditional loads (out-of-range entries read element 0 and are
      // replaced by zero) so that all of them are in flight together
      double2 v[NB];
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int idx = t + i * kInvThreads;
        const int rl = idx / NB, c = idx % NB;
        const bool ok = (r0 + rl < b) && (c < nbe);
        v[i] = A[ok ? (long long)(r0 + rl) * b + k0 + c : 0];
        if (!ok) v[i] = make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int idx = t + i * kInvThreads;
        stage[idx / NB][idx % NB] = v[i];
      }
      __syncthreads();
#pragma unroll
      for (int c = 0; c < NB; ++c) a[q][c] = stage[t][c];
      __syncthreads();
    } else {
#pragma unroll
      for (int c = 0; c < NB; ++c) a[q][c] = make_double2(0.0, 0.0);
    }
  }

  // Rows past b hold zeros and count as used, so they are never pivot
  // candidates and their elimination leaves them zero: no bounds tests in
  // the column loop.  Values read back from LDS are uniform across the
  // workgroup, so the failure bookkeeping branches uniformly.
  int first_bad = 0;
  int pv_reg[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    if (c >= nbe) continue;      // uniform across the workgroup
    const int par = c & 1;
    // ---- pivot search over unused rows -------------------------------
    double key = -1.0;
    int bad = 0;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int r = t + q * kInvThreads;
      if (!u[q]) {
        const double v = a[q][c].x * a[q][c].x + a[q][c].y * a[q][c].y;
        if (!(v <= 1.7976931348623157e308)) bad = 1;     // NaN or Inf
        else key = fmax(key, pivot_key(v, r));
      }
    }
    const double wk = wave_max(key);
    // the lane holding the wave's best candidate (keys are distinct) stores
    // that row for the other waves
    if (wk >= 0.0 && key == wk) {
      const int qs = (pivot_row(wk) - t) / kInvThreads;
#pragma unroll
      for (int q = 0; q < R; ++q)
        if (q == qs) {
#pragma unroll
          for (int cc = 0; cc < NB; ++cc) rowS[par][wave][cc] = a[q][cc];
        }
    }
    const int wbad = __any(bad);
    if (lane == 0) { keyS[par][wave] = wk; badS[par][wave] = wbad; }
    __syncthreads();
    double bk = keyS[par][0];
    int bw = 0, anybad = badS[par][0];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
      const double ok = keyS[par][w];
      if (ok > bk) { bk = ok; bw = w; }
      anybad |= badS[par][w];
    }
    // An unused row always remains (b - k0 - c > 0), so a candidate exists
    // unless every one was non-finite; then row 0 keeps indices in range
    // and the failure is reported through info.
    int p = (bk >= 0.0) ? pivot_row(bk) : 0;
    if (p >= b) p = 0;
    double2 prow[NB];
#pragma unroll
    for (int cc = 0; cc < NB; ++cc) prow[cc] = rowS[par][bw][cc];
    if (first_bad == 0) {
      const int code = code0 > 0 ? code0 : 1 + k0 + c;
      const double pv = prow[c].x * prow[c].x + prow[c].y * prow[c].y;
      if (anybad || bk < 0.0) first_bad = -code;
      else if (pv <= 0.0) first_bad = code;
    }
    pv_reg[c] = p;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const bool isp = (t + q * kInvThreads == p);
      u[q] |= isp;
      pc[q] = isp ? c : pc[q];
    }
    // ---- eliminate column k0 + c from every row ---------------------
    // every row as a non-pivot row, then the pivot row is replaced by the
    // scaled pivot row (its own update is discarded)
    const double2 inv = crecip_scaled(prow[c]);
    double2 ps[NB];
#pragma unroll
    for (int cc = 0; cc < NB; ++cc) ps[cc] = (cc == c) ? inv : cmul(prow[cc], inv);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      // a -= f * ps as four fused multiply-adds per element; column c
      // becomes -f * inv
      const double fx = a[q][c].x, fy = a[q][c].y;
#pragma unroll
      for (int cc = 0; cc < NB; ++cc) {
        const double2 z = (cc == c) ? make_double2(0.0, 0.0) : a[q][cc];
        a[q][cc].x = fma(-fx, ps[cc].x, fma(fy, ps[cc].y, z.x));
        a[q][cc].y = fma(-fx, ps[cc].y, fma(-fy, ps[cc].x, z.y));
      }
    }
#pragma unroll
    for (int q = 0; q < R; ++q)
      if (t + q * kInvThreads == p) {
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) a[q][cc] = ps[cc];
      }
  }
  if (t == 0) {
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < nbe) pivs[c] = pv_reg[c];
  }
  __syncthreads();                 // pivs[] complete before the write-back

  // ---- pivot rows within the super-panel (this panel's columns zeroed):
  // they lie outside the panel columns, so they are read before the panel
  // is written back
  constexpr int kG = NB * kSuper / kInvThreads;
  static_assert(NB * kSuper % kInvThreads == 0, "gather split");
  double2 gv[kG];
#pragma unroll
  for (int g = 0; g < kG; ++g) {
    const int idx = t + g * kInvThreads;
    const int c = idx / kSuper, j = lo + idx % kSuper;
    const int p = (c < nbe) ? pivs[c] : -1;
    const bool ok = (j < hi) && (p >= 0) && (j < k0 || j >= k0 + nbe);
    gv[g] = A[ok ? (long long)p * b + j : 0];
    if (!ok) gv[g] = make_double2(0.0, 0.0);
  }

  // ---- write back the panel and Panel'' (panel minus I at the pivots) ----
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int r0 = q * kInvThreads;
    if (r0 >= b) continue;                  // uniform across the workgroup
    if (r0 + t < b) ue[r0 + t] = u[q];
#pragma unroll
    for (int c = 0; c < NB; ++c) stage[t][c] = a[q][c];
    pcS[t] = pc[q];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int idx = t + i * kInvThreads;
      const int rl = idx / NB, c = idx % NB;
      const int r = r0 + rl;
      if (r < b) {
        double2 v = stage[rl][c];
        if (c < nbe) A[(long long)r * b + k0 + c] = v;
        if (pcS[rl] == c) v.x -= 1.0;
        pan[(long long)r * NB + c] = v;
      }
    }
    __syncthreads();
  }
  if (t < nbe) pe[k0 + t] = pivs[t];
  if (t == 0 && d.info) {
    // several inverses of one energy may share a launch (the partitions of
    // a partitioned solve): only a failure is written, so a success never
    // overwrites another inverse's failure
    int* inf = d.info + e;
    if (k0 == 0 && d.reset_info) *inf = first_bad;
    else if (first_bad != 0 && *inf == 0) *inf = first_bad;
  }
#pragma unroll
  for (int g = 0; g < kG; ++g) {
    const int idx = t + g * kInvThreads;
    const int c = idx / kSuper, j = lo + idx % kSuper;
    if (j < hi) br[(long long)c * b + j] = gv[g];
  }
}

// For the W-column panel at K0 (W = kSuper or kMega):
// spanel[r][c] = A[r][K0 + c] - (r == p_{K0+c}),  sbrow[c][j] = A[p_{K0+c}][j]
// outside [K0, K0 + W) and 0 inside; c beyond the matrix are zero.
__global__ __launch_bounds__(256)
void gj_super_gather_kernel(FlatLaunch L, int K0, int W) {
  const int di = find_desc(L.prefix, L.nd, blockIdx.x);
  const InvDesc& d = ((const InvDesc*)L.desc)[di];
  const int b = d.b;
  const int chunks = super_gather_chunks(b, W);
  const int local = blockIdx.x - L.prefix[di];
  const long long e = local / chunks;
  const long long q0 = (long long)(local % chunks) * kGatherItems;
  const double2* A = (const double2*)d.S + e * d.sS;
  const int* pe = d.perm + e * b;
  const int span = inv_span(b);
  double2* sp = (double2*)d.spanel + e * (long long)b * span;
  double2* sb = (double2*)d.sbrow + e * (long long)span * b;
  const int spe = min(W, b - K0);
  const long long half = (long long)b * W;
  const long long q1 = min(q0 + kGatherItems, 2 * half);
  for (long long q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
    if (q < half) {
      const int r = (int)(q / W), c = (int)(q % W);
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

hipError_t launch_inv_super_gather(int K0, int W, const FlatLaunch& l, hipStream_t s) {
  if (l.total <= 0) return hipSuccess;
  if (W != kSuper && W != kMega) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gj_super_gather_kernel, dim3(l.total), dim3(256), 0, s, l, K0, W);
  return hipGetLastError();
}

hipError_t launch_inv_permute(const FlatLaunch& l, hipStream_t s) {
  if (l.total <= 0) return hipSuccess;
  hipLaunchKernelGGL(gj_permute_kernel, dim3(l.total), dim3(256), 0, s, l);
  return hipGetLastError();
}

}  // namespace qtx
