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
//
// Matrices of at most kSmallB rows skip the blocking: one workgroup holds
// the whole matrix in registers and eliminates it column by column in a
// single launch (gj_small_kernel).
//
// Matrices above kInvThreads * 4 rows do not fit one workgroup's registers.
// Their panels pick the pivot rows by a tournament: every chunk of
// kTallChunk rows eliminates the panel columns on its own rows and proposes
// the rows it pivoted on; one workgroup eliminates the proposed rows, which
// fixes the panel's pivot rows p_0..p_15 and leaves on them the inverse of
// the pivot block B = A[p_k][k0 + j] (Gauss-Jordan on B); every other row r
// then becomes -A[r][panel] B^{-1}, the value the elimination would leave
// there.  This is the selection of communication-avoiding LU: it keeps the
// elimination stable in practice though its worst-case growth bound is
// weaker than that of partial pivoting over the whole column.
#include "qtx_internal.h"

namespace qtx {
namespace {

// Pivot search key of a candidate row r (< 1024) with |z|^2 = v (finite,
// >= 0): bits 62..42 of v (its exponent and top 10 mantissa bits) above the
// 10 bits of 1023 - r, plus one; 0 means no candidate.  Keys order as v to
// a relative 2^-10 and then by lowest row, so the largest key picks a pivot
// whose |z|^2 is within 0.1% of the column's largest (partial pivoting: the
// growth bound is that of the exact choice up to that factor) and names its
// row.  32-bit keys make the wave reduction one DPP max per step.
__device__ __forceinline__ unsigned pivot_key(double v, int r) {
  const unsigned hi = (unsigned)((unsigned long long)__double_as_longlong(v) >> 42);
  return ((hi << 10) | (unsigned)(1023 - r)) + 1u;
}
__device__ __forceinline__ int pivot_row(unsigned key) {
  return 1023 - (int)((key - 1u) & 1023u);
}

// x combined with its value in another lane moved by a DPP pattern (lanes
// of rows outside row_mask see 0, the identity of the unsigned maximum)
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned dpp_max(unsigned x) {
  const unsigned y = (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWS, 0xf, false);
  return x > y ? x : y;
}

// Maximum over the 64 lanes of a wave, returned in every lane: within rows
// of 16 lanes (quad xor 1, quad xor 2, half-row mirror, row mirror: every
// lane then holds its row's maximum), then lane 15 into rows 1 and 3 and
// lane 31 into rows 2 and 3, after which lane 63 holds the maximum.
__device__ __forceinline__ unsigned wave_max(unsigned x) {
  x = dpp_max<0xB1, 0xf>(x);     // quad_perm [1,0,3,2]
  x = dpp_max<0x4E, 0xf>(x);     // quad_perm [2,3,0,1]
  x = dpp_max<0x141, 0xf>(x);    // row_half_mirror
  x = dpp_max<0x140, 0xf>(x);    // row_mirror
  x = dpp_max<0x142, 0xa>(x);    // row_bcast:15
  x = dpp_max<0x143, 0xc>(x);    // row_bcast:31
  return (unsigned)__builtin_amdgcn_readlane((int)x, 63);
}

// 1/z without branches: z is scaled by an exact power of two so that
// d = |z'|^2 lies in [1/4, 2), then 1/z = conj(z') / d scaled back, with 1/d
// from the hardware reciprocal estimate refined by two Newton-Raphson steps
// r <- r + r (1 - d r), each of which squares the relative error (the
// estimate's is far below 2^-20, so the result is within a few ulp).  z = 0
// gives non-finite values; the caller flags that pivot.
__device__ __forceinline__ double2 crecip_scaled(double2 z) {
  const double s = fmax(fabs(z.x), fabs(z.y));
  int ex;
  (void)frexp(s, &ex);
  const double xr = ldexp(z.x, -ex), xi = ldexp(z.y, -ex);
  const double d = fma(xr, xr, xi * xi);
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  r = fma(r, fma(-d, r, 1.0), r);
  return make_double2(ldexp(xr * r, -ex), ldexp(-xi * r, -ex));
}

// a -= g * x (complex), four fused multiply-adds
__device__ __forceinline__ void axpy_neg(double2& a, double2 g, double2 x) {
  a.x = fma(-g.x, x.x, fma(g.y, x.y, a.x));
  a.y = fma(-g.x, x.y, fma(-g.y, x.x, a.y));
}

// This thread's best pivot key in panel column c over its unused rows
// (0 if none); bad is set for a non-finite candidate.
// Pins the computation of v where it stands: without it the compiler moves
// the reciprocal into the one lane that stores it, after the update it is
// meant to overlap.
__device__ __forceinline__ void keep(double2 v) { asm volatile("" ::"v"(v.x), "v"(v.y)); }

// A value written to LDS by one lane is read by the other lanes of its
// wave: LDS operations of a wave are performed in order, so only the
// compiler has to keep the read after the write.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int R>
__device__ __forceinline__ unsigned col_key(const double2 (&a)[R][kPanel], const int (&u)[R],
                                            int c, int t, int& bad) {
  unsigned key = 0;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    if (!u[q]) {
      const double v = a[q][c].x * a[q][c].x + a[q][c].y * a[q][c].y;
      if (!(v <= 1.7976931348623157e308)) bad = 1;     // NaN or Inf
      else {
        const unsigned k = pivot_key(v, t + q * kInvThreads);
        key = k > key ? k : key;
      }
    }
  }
  return key;
}

// The lane holding its wave's best candidate (keys are distinct) stores
// that row's element in column c, or the whole row.
template <int R>
__device__ __forceinline__ void publish_elem(const double2 (&a)[R][kPanel], unsigned key,
                                             unsigned wk, int c, int t, double2* dst) {
  if (wk != 0 && key == wk) {
    const int qs = (pivot_row(wk) - t) / kInvThreads;
#pragma unroll
    for (int q = 0; q < R; ++q)
      if (q == qs) *dst = a[q][c];
  }
}
template <int R>
__device__ __forceinline__ void publish_row(const double2 (&a)[R][kPanel], unsigned key,
                                            unsigned wk, int t, double2* dst) {
  if (wk != 0 && key == wk) {
    const int qs = (pivot_row(wk) - t) / kInvThreads;
#pragma unroll
    for (int q = 0; q < R; ++q)
      if (q == qs) {
#pragma unroll
        for (int cc = 0; cc < kPanel; ++cc) dst[cc] = a[q][cc];
      }
  }
}

// MODE 0: one workgroup per matrix factors the panel on all rows (b <= 4 *
// kInvThreads).  MODE 1: one workgroup per chunk of kTallChunk rows
// eliminates the panel on its rows and records the rows it pivoted on and
// which columns met a non-finite candidate.  MODE 2: one workgroup per
// matrix eliminates the recorded rows (the panel's pivot rows follow), and
// writes the inverse of the pivot block, the pivot rows, the status and the
// gathered pivot rows of the super-panel; gj_tall_apply_kernel does the rest.
template <int R, int MODE>
__global__ __launch_bounds__(kInvThreads)
void gj_panel_kernel(FlatLaunch L, int k0) {
  constexpr int NB = kPanel;
  constexpr int NW = kInvThreads / 64;
  // per column: each wave publishes its best key, that candidate's row and
  // the reciprocal of its pivot element; double buffered by column parity
  // so one barrier per column suffices
  __shared__ unsigned keyS[2][NW];
  __shared__ int badS[2][NW];
  __shared__ double2 rowS[2][NW][NB];
  __shared__ double2 invS[2][NW];   // reciprocal of the candidate's pivot element
  __shared__ double2 elemS[NW];     // the candidate's pivot element
  __shared__ double2 pinvS[NB];     // reciprocal pivot of each panel column
  __shared__ int pivs[NB];

  __shared__ int rowmap[kTallCand];  // MODE 2: the recorded rows
  const int di = find_desc(L.prefix, L.nd, blockIdx.x);
  const InvDesc& d = ((const InvDesc*)L.desc)[di];
  const int b = d.b;
  const int local = blockIdx.x - L.prefix[di];
  const int nch = tall_chunks(b);
  const int e = MODE == 1 ? local / nch : local;
  const int ch = MODE == 1 ? local % nch : 0;
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
  // the workgroup's rows: local row i is matrix row grow(i), i < nrows
  int* tc = tall_cand(d, e, b);                    // MODE 1/2 records
  const int base = ch * kTallChunk;
  const int nrows = MODE == 0 ? b : MODE == 1 ? min(kTallChunk, b - base) : nch * NB;
  unsigned tbad = 0;                               // MODE 2: columns flagged by a chunk
  if (MODE == 2) {
    for (int i = t; i < kTallCand; i += kInvThreads) rowmap[i] = i < nrows ? tc[i] : -1;
    for (int j = 0; j < nch; ++j) tbad |= (unsigned)tc[kTallCand + j];
    __syncthreads();
  }
  auto grow = [&](int i) { return MODE == 0 ? i : MODE == 1 ? base + i : rowmap[i]; };

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
    if (r < nrows) {
      if (MODE == 2) u[q] = grow(r) >= 0 ? 0 : 1;   // recorded rows are unused
      else u[q] = (k0 == 0) ? 0 : ue[grow(r)];
    }
    if (r0 < nrows) {                       // uniform across the workgroup
      // unconditional loads (out-of-range entries read element 0 and are
      // replaced by zero) so that all of them are in flight together
      double2 v[NB];
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int idx = t + i * kInvThreads;
        const int rl = idx / NB, c = idx % NB;
        const int gr = (r0 + rl < nrows) ? grow(r0 + rl) : -1;
        const bool ok = (gr >= 0) && (c < nbe);
        v[i] = A[ok ? (long long)gr * b + k0 + c : 0];
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
  //
  // Pivot rows are left unscaled while the panel is eliminated: the row
  // chosen for column c keeps its values with 1 in column c, and the later
  // eliminations (linear in the row) act on it unchanged, so scaling it by
  // the reciprocal pivot once after the last column gives the same panel.
  // Non-pivot rows take the multiplier g = a[r][c] / pivot.  Column c + 1 is
  // updated first: its pivot search, and the reciprocal of each wave's
  // candidate (read back through LDS by the whole wave), then overlap the
  // update of the other columns.
  int first_bad = 0;
  int pv_reg[NB];
  unsigned hcm = 0, hbm = 0;     // MODE 1: columns with a candidate / a non-finite one
  {
    int bad = 0;
    const unsigned key = col_key<R>(a, u, 0, t, bad);
    const unsigned wk = wave_max(key);
    publish_elem<R>(a, key, wk, 0, t, &elemS[wave]);
    wave_sync();
    const double2 inv0 = crecip_scaled(elemS[wave]);   // stale (unused) without a candidate
    publish_row<R>(a, key, wk, t, rowS[0][wave]);
    const int wbad = __any(bad);
    if (lane == 0) { keyS[0][wave] = wk; badS[0][wave] = wbad; invS[0][wave] = inv0; }
  }
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    if (c >= nbe) continue;      // uniform across the workgroup
    const int par = c & 1;
    __syncthreads();
    unsigned bk = keyS[par][0];
    int bw = 0, anybad = badS[par][0];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
      const unsigned ok = keyS[par][w];
      if (ok > bk) { bk = ok; bw = w; }
      anybad |= badS[par][w];
    }
    // An unused row always remains (b - k0 - c > 0), so a candidate exists
    // unless every one was non-finite; then row 0 keeps indices in range
    // and the failure is reported through info.
    int p = bk ? pivot_row(bk) : 0;
    if (p >= nrows) p = 0;
    // A chunk (MODE 1) whose remaining rows are all zero in this column (or
    // none is left) skips it: it proposes no row for it and eliminates
    // nothing, so its proposals stay a basis of its rows' panel entries.
    const bool skip = MODE == 1 && (bk == 0 || ((bk - 1u) >> 10) == 0);
    if (MODE == 1 && !skip) hcm |= 1u << c;
    if (MODE == 1 && anybad) hbm |= 1u << c;
    if (MODE == 2) anybad |= (tbad >> c) & 1u;
    // what the multipliers and column c + 1 need is read first
    const double2 inv = invS[par][bw];
    // (the winning wave as a scalar, so that the 16 reads share one
    // address register and differ in their offsets)
    const double2* src = &rowS[par][0][0] + __builtin_amdgcn_readfirstlane(bw) * NB;
    double2 prow[NB];
    if (c + 1 < NB) prow[c + 1] = src[c + 1];
    prow[c] = src[c];
#pragma unroll
    for (int cc = 0; cc < NB; ++cc)
      if (cc != c && cc != c + 1) prow[cc] = src[cc];
    {
      const int code = code0 > 0 ? code0 : 1 + k0 + c;
      const double pv = prow[c].x * prow[c].x + prow[c].y * prow[c].y;
      const int st = (anybad || bk == 0) ? -code : (pv <= 0.0 ? code : 0);
      first_bad = first_bad != 0 ? first_bad : st;
    }
    pv_reg[c] = p;
    // multipliers; the pivot row takes none (it stays as it is)
    bool isp[R];
    double2 g[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      isp[q] = !skip && (t + q * kInvThreads == p);
      u[q] |= isp[q];
      pc[q] = isp[q] ? c : pc[q];
      const double2 m = cmul(a[q][c], inv);
      g[q] = (isp[q] || skip) ? make_double2(0.0, 0.0) : m;
    }
    // ---- column c + 1 first, and the next pivot search
    const bool nxt = c + 1 < nbe;  // uniform across the workgroup
    unsigned key1 = 0, wk1 = 0;
    int bad1 = 0;
    if (c + 1 < NB) {
#pragma unroll
      for (int q = 0; q < R; ++q) axpy_neg(a[q][c + 1], g[q], prow[c + 1]);
      if (nxt) {
        key1 = col_key<R>(a, u, c + 1, t, bad1);
        wk1 = wave_max(key1);
        publish_elem<R>(a, key1, wk1, c + 1, t, &elemS[wave]);
      }
    }
    // outside the branch, so that it interleaves with the update below
    // (without a next column it reads a stale element and is not used)
    wave_sync();
    const double2 inv1 = crecip_scaled(elemS[wave]);
    keep(inv1);
    // ---- the other columns
#pragma unroll
    for (int cc = 0; cc < NB; ++cc) {
      if (cc == c || cc == c + 1) continue;
#pragma unroll
      for (int q = 0; q < R; ++q) axpy_neg(a[q][cc], g[q], prow[cc]);
    }
#pragma unroll
    for (int q = 0; q < R; ++q)
      a[q][c] = isp[q] ? make_double2(1.0, 0.0) : make_double2(-g[q].x, -g[q].y);
    if (c + 1 < NB && nxt) {
      publish_row<R>(a, key1, wk1, t, rowS[par ^ 1][wave]);
      const int wbad = __any(bad1);
      if (lane == 0) {
        keyS[par ^ 1][wave] = wk1;
        badS[par ^ 1][wave] = wbad;
        invS[par ^ 1][wave] = inv1;
      }
    }
    if (t == 0) pinvS[c] = inv;
  }
  if (MODE == 1) {
    // the rows this chunk pivoted on, and its flags of non-finite columns
    if (t == 0) {
      int* rec = tc + ch * NB;
#pragma unroll
      for (int c = 0; c < NB; ++c)
        rec[c] = (c < nbe && ((hcm >> c) & 1u)) ? base + pv_reg[c] : -1;
      tc[kTallCand + ch] = (int)hbm;
    }
    return;
  }
  if (t == 0) {
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < nbe) pivs[c] = grow(pv_reg[c]);
  }
  __syncthreads();                 // pivs[], pinvS[] complete

  // ---- scale the pivot rows by their reciprocal pivots
#pragma unroll
  for (int q = 0; q < R; ++q) {
    if (pc[q] >= 0) {
      const double2 s = pinvS[pc[q]];
#pragma unroll
      for (int cc = 0; cc < NB; ++cc)
        if (cc < nbe) a[q][cc] = cmul(a[q][cc], s);
    }
  }

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

  if (MODE == 2) {
    // row k of the pivot block's inverse is left on pivot row k (rows past
    // the panel's width are zero)
    double2* binv = tall_binv(d, e, b);
#pragma unroll
    for (int q = 0; q < R; ++q)
      if (pc[q] >= 0) {
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) binv[pc[q] * NB + cc] = a[q][cc];
      }
    for (int i = nbe * NB + t; i < NB * NB; i += kInvThreads) binv[i] = make_double2(0.0, 0.0);
  }
  // ---- write back the panel and Panel'' (panel minus I at the pivots) ----
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int r0 = q * kInvThreads;
    if (MODE != 0) continue;
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

// The tournament path's last step for the panel at k0: row r becomes row k
// of the pivot block's inverse if it is pivot row p_k, else -A[r][panel]
// times that inverse; Panel'' and the used flags follow.  Rows move through
// LDS as in the panel kernel (16 lanes per row in HBM).
__global__ __launch_bounds__(kInvThreads)
void gj_tall_apply_kernel(FlatLaunch L, int k0) {
  constexpr int NB = kPanel;
  __shared__ double2 binvS[NB][NB];
  __shared__ int pivS[NB];
  __shared__ double2 stage[kInvThreads][NB + 1];
  __shared__ int pcS[kInvThreads];
  const int di = find_desc(L.prefix, L.nd, blockIdx.x);
  const InvDesc& d = ((const InvDesc*)L.desc)[di];
  const int b = d.b;
  const int nblk = (b + kInvThreads - 1) / kInvThreads;
  const int local = blockIdx.x - L.prefix[di];
  const int e = local / nblk;
  const int r0 = (local % nblk) * kInvThreads;
  if (k0 >= b) return;
  const int t = threadIdx.x;
  const int nbe = min(NB, b - k0);
  double2* A = (double2*)d.S + e * d.sS;
  const int* pe = d.perm + (long long)e * b;
  int* ue = d.used + (long long)e * b;
  double2* pan = (double2*)d.panel + (long long)e * b * NB;
  const double2* binv = tall_binv(d, e, b);
  for (int i = t; i < NB * NB; i += kInvThreads) binvS[i / NB][i % NB] = binv[i];
  if (t < NB) pivS[t] = t < nbe ? pe[k0 + t] : -1;
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
  double2 a[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) a[c] = stage[t][c];
  const int r = r0 + t;
  int k = -1;
#pragma unroll
  for (int j = 0; j < NB; ++j) k = (pivS[j] == r) ? j : k;
  double2 y[NB];
  if (k >= 0) {
#pragma unroll
    for (int j = 0; j < NB; ++j) y[j] = binvS[k][j];
  } else {
#pragma unroll
    for (int j = 0; j < NB; ++j) y[j] = make_double2(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < NB; ++i) {
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const double2 m = binvS[i][j];
        y[j].x = fma(-a[i].x, m.x, fma(a[i].y, m.y, y[j].x));
        y[j].y = fma(-a[i].x, m.y, fma(-a[i].y, m.x, y[j].y));
      }
    }
  }
  if (r < b) ue[r] = ((k0 == 0) ? 0 : ue[r]) | (k >= 0 ? 1 : 0);
  __syncthreads();                  // stage is reused
#pragma unroll
  for (int c = 0; c < NB; ++c) stage[t][c] = y[c];
  pcS[t] = k;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int idx = t + i * kInvThreads;
    const int rl = idx / NB, c = idx % NB;
    const int rr = r0 + rl;
    if (rr < b) {
      double2 w = stage[rl][c];
      if (c < nbe) A[(long long)rr * b + k0 + c] = w;
      if (pcS[rl] == c) w.x -= 1.0;
      pan[(long long)rr * NB + c] = w;
    }
  }
}

// X[k][c] = Y[p_k][pinv(c)] with pinv(p_j) = j; kPermRows rows per workgroup.
__global__ __launch_bounds__(256)
void gj_permute_kernel(FlatLaunch L) {
  __shared__ int pinv[kMaxB];
  __shared__ int pk[kMaxB];
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

// ---- the whole inverse in one workgroup (b <= kSmallB) ----------------------
//
// A matrix of up to 16 TR rows fits the registers of one workgroup of TR
// waves.  Wave w holds columns [16 w, 16 w + 16); lane 16 ct + rt of it
// holds a tile of rows rt + 16 i (i < TR) by columns 16 w + 4 ct + j
// (j < 4).  The columns are eliminated one at a time in one launch, so the
// inverse is one launch instead of a chain of panels and updates.  Per
// column k, with one barrier: every wave reads the pivot row p_k and the
// reciprocal pivot published for it, takes the pivot row's entries in its
// columns from the four lanes that hold them (through LDS, within the
// wave), forms the multipliers g_r = A[r][k] / pivot of its rows from the
// published column and applies the rank-1 update to its tile.  The wave
// holding column k + 1 updates that column first, searches it for the next
// pivot row (a maximum over the column's 16 lanes) and publishes the
// column and the reciprocal of its pivot, which overlaps the other waves'
// updates.  The tile shape keeps what each lane reads per column to 4
// pivot-row entries and TR column entries.  (Measured slower: a 16-column
// panel eliminated inside one wave with the other columns updated once per
// panel, where the other waves idle while the panel's columns go one after
// the other; and the winner's reciprocal taken by readlane from every
// lane's own candidate, which lengthens the search.)
//
// Pivot rows are left unscaled until all columns are done (as in the panel
// kernel), and each eliminated column holds +g_r with -1 on its pivot row,
// the negative of the Gauss-Jordan column (-g_r, and 1 before the
// deferred scaling).  Later updates are linear in every eliminated column,
// so the whole result comes out negated, and the final scaling of pivot
// row p_k by -1/pivot_k undoes that; negation is exact, so the result has
// the bits of the unnegated elimination.  The published column carries a
// zero on the pivot row, which therefore takes no multiplier.  The result
// is written permuted, X[k][p_j] = Y[p_k][j], through LDS in passes of 64
// rows so that the stores are coalesced.
template <int TR>
__global__ __launch_bounds__(64 * TR)
void gj_small_kernel(FlatLaunch L) {
  constexpr int SB = 16 * TR;           // largest b: rows and columns
  constexpr int NW = SB / 16;           // waves, 16 columns each
  constexpr int NT = 64 * NW;           // threads
  __shared__ uint2 hdrS[2];             // by column parity: pivot key, flags (1 non-finite, 2 zero pivot)
  __shared__ double2 invS[2];           // reciprocal of the pivot
  __shared__ double2 colS[2][4][SB];    // the column at each lane column offset of the searching wave
  __shared__ double2 rowW[NW][16];      // the pivot row's entries in each wave's columns
  __shared__ int permS[SB];             // pivot row of each column
  __shared__ int posS[SB];              // column that row r pivots
  __shared__ double2 pinvS[SB];         // reciprocal pivot of each column
  __shared__ double2 stage[64][SB + 1]; // 64 rows on their way to or from HBM

  const int di = find_desc(L.prefix, L.nd, blockIdx.x);
  const InvDesc& d = ((const InvDesc*)L.desc)[di];
  const int b = d.b;
  const long long e = blockIdx.x - L.prefix[di];
  const double2* A = (const double2*)d.S + e * d.sS;
  double2* X = (double2*)d.X + e * d.sX;
  const int code0 = d.code;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int rt = lane & 15, ct = lane >> 4;
  const int cb = 16 * wave + 4 * ct;    // this lane's first column

  double2 a[TR][4];
  for (int i = t; i < SB; i += NT) posS[i] = i;
#pragma unroll
  for (int q = 0; q < TR / 4; ++q) {
    // rows [64 q, 64 q + 64), i.e. rows rt + 16 i for i in [4 q, 4 q + 4):
    // coalesced into LDS, then each lane takes its tile (zero past b)
#pragma unroll
    for (int s = 0; s < 64 * SB / NT; ++s) {
      const int idx = t + s * NT;
      const int rl = idx / SB, c = idx % SB;
      const int r = 64 * q + rl;
      const bool ok = r < b && c < b;
      double2 v = A[ok ? (long long)r * b + c : 0];
      if (!ok) v = make_double2(0.0, 0.0);
      stage[rl][c] = v;
    }
    __syncthreads();
#pragma unroll
    for (int ii = 0; ii < 4; ++ii)
#pragma unroll
      for (int j = 0; j < 4; ++j) a[4 * q + ii][j] = stage[rt + 16 * ii][cb + j];
    __syncthreads();
  }
  unsigned um = 0;                      // bit i: row rt + 16 i already a pivot row (rows past b count as used)
#pragma unroll
  for (int i = 0; i < TR; ++i) um |= (rt + 16 * i >= b ? 1u : 0u) << i;

  // Search of column 16 w + 4 nct + nj (register column nj of the lanes
  // with ct == nct) over the unused rows; all lanes' register column nj goes
  // to colS[buf][ct], and the winner's key, the non-finite flag, the pivot
  // row and the pivot element come back uniform.
  auto search = [&](int nj, int nct, int buf, unsigned& wk, int& wbad, int& pn,
                    double2& pe) __attribute__((always_inline)) {
    unsigned key = 0;
    int bad = 0;
#pragma unroll
    for (int i = 0; i < TR; ++i) {
      const double v = a[i][nj].x * a[i][nj].x + a[i][nj].y * a[i][nj].y;
      const bool fin = v <= 1.7976931348623157e308;     // not NaN or Inf
      const bool un = ((um >> i) & 1u) == 0;
      bad |= (un && !fin) ? 1 : 0;
      const unsigned kv = (un && fin) ? pivot_key(v, rt + 16 * i) : 0u;
      key = kv > key ? kv : key;
    }
    // maximum over each row of 16 lanes (the first four steps of wave_max)
    key = dpp_max<0xB1, 0xf>(key);
    key = dpp_max<0x4E, 0xf>(key);
    key = dpp_max<0x141, 0xf>(key);
    key = dpp_max<0x140, 0xf>(key);
    wk = (unsigned)__builtin_amdgcn_readlane((int)key, 16 * nct);
    wbad = __any(bad != 0 && ct == nct);
#pragma unroll
    for (int i = 0; i < TR; ++i) colS[buf][ct][rt + 16 * i] = a[i][nj];
    wave_sync();
    pn = wk ? pivot_row(wk) : 0;
    pn = pn < SB ? pn : 0;
    pe = colS[buf][nct][pn];
  };
  // After the search's wave has done its update: the header, the
  // reciprocal pivot and a zero on the pivot row of the published column.
  auto publish = [&](int nct, int buf, unsigned wk, int wbad, int pn, double2 pe,
                     double2 inv1) __attribute__((always_inline)) {
    if (lane == 0) {
      const double pv = pe.x * pe.x + pe.y * pe.y;
      hdrS[buf] = make_uint2(wk, (wbad ? 1u : 0u) | (pv <= 0.0 ? 2u : 0u));
      invS[buf] = inv1;
      colS[buf][nct][pn] = make_double2(0.0, 0.0);
    }
  };
  if (wave == 0) {
    unsigned wk;
    int wbad, pn;
    double2 pe;
    search(0, 0, 0, wk, wbad, pn, pe);
    publish(0, 0, wk, wbad, pn, pe, crecip_scaled(pe));
  }

  int first_bad = 0;
  for (int kk = 0; kk < b; kk += 16) {
    const int G = kk >> 4;              // the wave holding columns kk .. kk + 15
#pragma unroll
    for (int cl = 0; cl < 16; ++cl) {
      const int k = kk + cl;
      if (k >= b) continue;             // uniform across the workgroup
      const int par = cl & 1;
      const int ctk = cl >> 2, jk = cl & 3;   // lanes and register column of column k in wave G
      __syncthreads();
      const uint2 hd = hdrS[par];
      const double2 inv = invS[par];
      // A candidate exists unless every unused row was non-finite in this
      // column; then row 0 keeps indices in range and info reports it.
      int p = hd.x ? pivot_row(hd.x) : 0;
      if (p >= b) p = 0;
      const int ip = __builtin_amdgcn_readfirstlane(p >> 4), rtp = p & 15;
      if (rt == rtp) {
#pragma unroll
        for (int i = 0; i < TR; ++i)
          if (i == ip) {
#pragma unroll
            for (int j = 0; j < 4; ++j) rowW[wave][4 * ct + j] = a[i][j];
          }
      }
      wave_sync();
      double2 prow[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) prow[j] = rowW[wave][4 * ct + j];
      {
        const int code = code0 > 0 ? code0 : 1 + k;
        const int st = ((hd.y & 1u) || hd.x == 0) ? -code : ((hd.y & 2u) ? code : 0);
        first_bad = first_bad != 0 ? first_bad : st;
      }
      if (t == 0) { permS[k] = p; pinvS[k] = inv; }
      double2 g[TR];
#pragma unroll
      for (int i = 0; i < TR; ++i) {
        g[i] = cmul(colS[par][ctk][rt + 16 * i], inv);
        um |= (rt + 16 * i == p ? 1u : 0u) << i;
      }
      // column k in the lanes holding it: +g, and -1 on the pivot row (where g is 0)
      const bool ownk = wave == G && ct == ctk;
      const int nj = (cl + 1) & 3, nct = ((cl + 1) & 15) >> 2;
      const int nwave = cl + 1 < 16 ? G : G + 1;
      if (wave == nwave && k + 1 < b) {   // uniform across the wave
#pragma unroll
        for (int i = 0; i < TR; ++i) axpy_neg(a[i][nj], g[i], prow[nj]);
        unsigned wk;
        int wbad, pn;
        double2 pe;
        search(nj, nct, par ^ 1, wk, wbad, pn, pe);
        const double2 inv1 = crecip_scaled(pe);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (j == nj) continue;
#pragma unroll
          for (int i = 0; i < TR; ++i) axpy_neg(a[i][j], g[i], prow[j]);
        }
#pragma unroll
        for (int i = 0; i < TR; ++i) {
          const double2 h = make_double2(g[i].x + (rt + 16 * i == p ? -1.0 : 0.0), g[i].y);
          if (ownk) a[i][jk] = h;      // (a store, not a select of two lvalues: that would take their addresses)
        }
        publish(nct, par ^ 1, wk, wbad, pn, pe, inv1);
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int i = 0; i < TR; ++i) axpy_neg(a[i][j], g[i], prow[j]);
#pragma unroll
        for (int i = 0; i < TR; ++i) {
          const double2 h = make_double2(g[i].x + (rt + 16 * i == p ? -1.0 : 0.0), g[i].y);
          if (ownk) a[i][jk] = h;      // (a store, not a select of two lvalues: that would take their addresses)
        }
      }
    }
  }
  __syncthreads();                      // permS, pinvS complete
  // Pivots are distinct rows unless a non-finite column was met (flagged
  // through info); rows named twice keep every index in range.
  for (int k = t; k < b; k += NT) posS[permS[k]] = k;
  __syncthreads();
  int pc[4];                            // destination column of each register column
#pragma unroll
  for (int j = 0; j < 4; ++j) pc[j] = cb + j < b ? permS[cb + j] : -1;
#pragma unroll
  for (int q2 = 0; q2 < TR / 4; ++q2) {
    // destination rows [64 q2, 64 q2 + 64); row r goes to row posS[r],
    // scaled by minus its reciprocal pivot
#pragma unroll
    for (int i = 0; i < TR; ++i) {
      const int r = rt + 16 * i;
      const int pr = r < b ? posS[r] : -1;
      if (pr >= 0 && pr >> 6 == q2) {
        const double2 s = pinvS[pr];
        const double2 ns = make_double2(-s.x, -s.y);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (pc[j] >= 0) stage[pr & 63][pc[j]] = cmul(a[i][j], ns);
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 64 * SB / NT; ++s) {
      const int idx = t + s * NT;
      const int rl = idx / SB, c = idx % SB;
      const int r = 64 * q2 + rl;
      if (r < b && c < b) X[(long long)r * b + c] = stage[rl][c];
    }
    __syncthreads();
  }
  if (t == 0 && d.info) {
    int* inf = d.info + e;
    if (d.reset_info) *inf = first_bad;
    else if (first_bad != 0 && *inf == 0) *inf = first_bad;
  }
}

}  // namespace

hipError_t launch_inv_small(int rpl, const FlatLaunch& l, hipStream_t s) {
  if (l.total <= 0) return hipSuccess;
  switch (rpl) {
    case 1: hipLaunchKernelGGL((gj_small_kernel<4>), dim3(l.total), dim3(256), 0, s, l); break;
    case 2: hipLaunchKernelGGL((gj_small_kernel<8>), dim3(l.total), dim3(512), 0, s, l); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_inv_panel(int R, int k0, const FlatLaunch& l, hipStream_t s) {
  if (l.total <= 0) return hipSuccess;
  switch (R) {
    case 1: hipLaunchKernelGGL((gj_panel_kernel<1, 0>), dim3(l.total), dim3(kInvThreads), 0, s, l, k0); break;
    case 2: hipLaunchKernelGGL((gj_panel_kernel<2, 0>), dim3(l.total), dim3(kInvThreads), 0, s, l, k0); break;
    case 3: hipLaunchKernelGGL((gj_panel_kernel<3, 0>), dim3(l.total), dim3(kInvThreads), 0, s, l, k0); break;
    case 4: hipLaunchKernelGGL((gj_panel_kernel<4, 0>), dim3(l.total), dim3(kInvThreads), 0, s, l, k0); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_inv_tall(int step, int k0, const FlatLaunch& l, hipStream_t s) {
  if (l.total <= 0) return hipSuccess;
  static_assert(kTallChunk == 3 * kInvThreads, "chunk rows = 3 per thread");
  static_assert(kTallCand <= kInvThreads, "one recorded row per thread");
  switch (step) {
    case 1: hipLaunchKernelGGL((gj_panel_kernel<3, 1>), dim3(l.total), dim3(kInvThreads), 0, s, l, k0); break;
    case 2: hipLaunchKernelGGL((gj_panel_kernel<1, 2>), dim3(l.total), dim3(kInvThreads), 0, s, l, k0); break;
    case 3: hipLaunchKernelGGL(gj_tall_apply_kernel, dim3(l.total), dim3(kInvThreads), 0, s, l, k0); break;
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
