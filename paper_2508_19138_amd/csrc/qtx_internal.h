// Internal interfaces of the RGF library: the device descriptors that drive
// every kernel, and the launchers.  Not part of the public C ABI.
//
// Every kernel is descriptor-driven: a launch covers a table of descriptors
// in device memory, each describing a strided family of independent b x b
// block operations (one per energy and, optionally, per block index).  The
// grid is flat; workgroup w finds its descriptor by a binary search over an
// exclusive prefix sum of workgroups per descriptor.  One launch can thus
// serve many independent solves of different block size and block count.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qtx_device.h"

namespace qtx {

// Flat launch over `nd` descriptors of type T: workgroups
// [prefix[d], prefix[d+1]) belong to descriptor d; total = prefix[nd].
struct FlatLaunch {
  const void* desc;     // device, nd descriptors
  const int* prefix;    // device, nd + 1 entries
  int nd;
  int total;
};

// ---- complex products on the matrix cores ----------------------------------
// D[e,j] = alpha * op(A[e,j]) op(B[e,j]) + beta * C[e,j], e < batch,
// j < batch2; operand X[e,j] starts at X + e * sX + j * tX (complex128
// elements).  op(A) is M x K, op(B) is K x N.  C may be null (beta ignored)
// and may equal D.
struct GemmDesc {
  const void* A;
  const void* B;
  const void* C;
  void* D;
  long long sA, sB, sC, sD;
  long long tA, tB, tC, tD;
  long long lda, ldb, ldc, ldd;
  zc alpha, beta;
  int M, N, K;
  int batch, batch2;
  int tiles;            // workgroups per matrix (set by the launcher's config)
  // asm != 0 (C null, batch2 1, square blocks): the C term is assembled in
  // the epilogue, C[e] = (i0 + i1 E[e]) I + sum_t (xc_t + xd_t E[e]) X_t[e],
  // X_t[e] at X_t + e * sX_t (ld ldc; null terms skipped) -- the diagonal
  // block E S - H - Sigma^R formed where the Schur update is written
  int asm_;
  const void* X[3];
  long long sX[3];
  zc xc[3], xd[3];
  zc i0, i1;
  const double* E;
};

// Tile configurations of the product kernel (see zgemm.hip); the extra
// value kGemmInvUpdate selects the small tile under its own kernel symbol
// for the inverse's update products (FP64, N x N only; measured faster than
// the larger tiles for these thin or short products at any batch size).
constexpr int kGemmConfigs = 3;
constexpr int kGemmInvUpdate = 7;
int gemm_tile_m(int cfg);   // kGemmInvUpdate: the update tile; kGemmMegaUpdate: configuration 0
int gemm_tile_n(int cfg);
inline int gemm_tiles(int cfg, int M, int N) {
  return ((M + gemm_tile_m(cfg) - 1) / gemm_tile_m(cfg)) *
         ((N + gemm_tile_n(cfg) - 1) / gemm_tile_n(cfg));
}
// fp32 = false: FP64 matrix cores on complex128.  fp32 = true: operands
// rounded to complex64, FP32 matrix cores, FP64 epilogue.
hipError_t launch_gemm(int cfg, bool fp32, char opa, char opb,
                       const FlatLaunch& l, hipStream_t s);

// ---- Gauss-Jordan inverse with partial pivoting -----------------------------
constexpr int kPanel = 16;     // columns factored per panel step
constexpr int kSuper = 64;     // columns per super-panel
constexpr int kMega = 256;     // columns per mega-panel (three-level blocking)
constexpr int kInvThreads = 256;
// Columns of the gathered panel buffers (spanel, sbrow) per matrix: the
// super-panel width, or the mega-panel width when the matrix has more than
// one mega-panel (the two levels use the buffers one after the other).
__host__ __device__ inline int inv_span(int b) { return b > kMega ? kMega : kSuper; }

// `batch` matrices S[e] (b x b, stride sS) are eliminated in place; the
// inverses go to X[e] (stride sX).  Per-matrix work buffers (element strides
// in brackets): panel [b*kPanel], brow [kPanel*b], spanel [b*inv_span(b)],
// sbrow [inv_span(b)*b] (complex128), perm [b], used [b] (int).
// info[e]: 0, or set once to +code (zero pivot) / -code (non-finite pivot);
// `reset_info` clears it at the first panel.  code <= 0 means 1 + column.
struct InvDesc {
  void* S;
  void* X;
  long long sS, sX;
  void* panel;
  void* brow;
  void* spanel;
  void* sbrow;
  int* perm;
  int* used;
  int* info;
  int code;
  int reset_info;
  int b;
  int batch;
};
// Largest block size of the inverse.  Above kInvThreads * 4 rows the panel
// takes the tournament path (zinv.hip): chunks of kTallChunk rows propose
// pivot rows, at most kTallCand of them.
constexpr int kMaxB = 4096;
constexpr int kTallB = 4 * kInvThreads;
constexpr int kTallChunk = 3 * kInvThreads;
constexpr int kTallCand = (kMaxB + kTallChunk - 1) / kTallChunk * kPanel;
__host__ __device__ inline int tall_chunks(int b) { return (b + kTallChunk - 1) / kTallChunk; }
// The tournament path's records of matrix e, kept in its spanel buffer
// (which only the gather after a super-panel and the product reading it
// use): the pivot block's inverse [kPanel][kPanel], then the proposed rows
// [kTallCand] and each chunk's flags of non-finite columns [chunks].
__host__ __device__ inline double2* tall_binv(const InvDesc& d, long long e, int b) {
  return (double2*)d.spanel + e * (long long)b * inv_span(b);
}
__host__ __device__ inline int* tall_cand(const InvDesc& d, long long e, int b) {
  return (int*)(tall_binv(d, e, b) + kPanel * kPanel);
}
// Bytes of inverse work buffers per matrix of size b.
inline size_t inv_work_bytes(int b) {
  return (size_t)b * (2 * kPanel + 2 * inv_span(b)) * 16 + (size_t)b * 8;
}
// Panel factorisation of columns [k0, k0 + kPanel) of every matrix with
// b > k0 (one workgroup per matrix); R = rows per thread, b <= 256 R.  The
// pivot rows are gathered into brow for the columns [k0 & ~(kSuper-1),
// + kSuper) of the current super-panel.
hipError_t launch_inv_panel(int R, int k0, const FlatLaunch& l, hipStream_t s);
// The tournament path's three launches for the panel at k0 of matrices with
// b > kTallB: step 1 one workgroup per chunk of kTallChunk rows (proposals),
// step 2 one per matrix (pivot rows, pivot block inverse, status, gathered
// pivot rows), step 3 one per kInvThreads rows (every row of the panel,
// Panel'', used flags).
hipError_t launch_inv_tall(int step, int k0, const FlatLaunch& l, hipStream_t s);
// After the last panel of the W-column panel (W = kSuper or kMega) starting
// at K0: spanel = its eliminated columns minus the identity at their pivot
// rows [b][W], sbrow = its pivot rows outside it (zero inside) [W][b].
constexpr int kGatherItems = 2048;   // elements per workgroup
hipError_t launch_inv_super_gather(int K0, int W, const FlatLaunch& l, hipStream_t s);
__host__ __device__ inline int super_gather_chunks(int b, int W) {
  return (int)((2LL * b * W + kGatherItems - 1) / kGatherItems);
}
// Tile of the inverse's update products (the kGemmInvUpdate configuration).
constexpr int kInvUpdTile = 32;
// The rank-kMega updates run the recursion's product kernel (the 3M form,
// tiles of kMegaTile) under their own kernel symbol (configuration value
// kGemmMegaUpdate).
constexpr int kGemmMegaUpdate = 8;
constexpr int kMegaCfg = kGemmMegaUpdate;
constexpr int kMegaTile = 64;

// Update products of the blocked inverse, shared by every launcher of the
// inverse (host) and by the device-side descriptor set-up of the
// allocation-free entry point: the rank-kPanel update of the rest of the
// super-panel after the panel at column k0 (false: nothing left to update),
// and the rank-kSuper update of the whole matrix after the super-panel at
// K0 (false: the matrix has a single super-panel or ends before K0).
__host__ __device__ inline int inv_update_tiles(int M, int N) {
  return ((M + kInvUpdTile - 1) / kInvUpdTile) * ((N + kInvUpdTile - 1) / kInvUpdTile);
}
__host__ __device__ inline bool inv_panel_update(const InvDesc& v, int k0, GemmDesc* out) {
  const int K0 = k0 - k0 % kSuper;
  const int hi = v.b < K0 + kSuper ? v.b : K0 + kSuper;
  const int nbe = kPanel < v.b - k0 ? kPanel : v.b - k0;
  if (k0 >= v.b || hi - K0 <= nbe) return false;
  GemmDesc g{};
  g.M = v.b; g.N = hi - K0; g.K = kPanel;
  g.A = v.panel; g.sA = (long long)v.b * kPanel; g.lda = kPanel;
  g.B = (double2*)v.brow + K0; g.sB = (long long)kPanel * v.b; g.ldb = v.b;
  g.C = (double2*)v.S + K0; g.sC = v.sS; g.ldc = v.b;
  g.D = (double2*)v.S + K0; g.sD = v.sS; g.ldd = v.b;
  g.alpha = zc{1.0, 0.0};
  g.beta = zc{1.0, 0.0};
  g.batch = v.batch; g.batch2 = 1;
  g.tiles = inv_update_tiles(g.M, g.N);
  *out = g;
  return true;
}
// The rank-kSuper update after the super-panel at K0 covers the columns of
// its mega-panel [M0, Mend) only (all of them when b <= kMega): the columns
// of later mega-panels take the whole mega-panel's eliminations at once.
__host__ __device__ inline bool inv_super_update(const InvDesc& v, int K0, GemmDesc* out) {
  if (v.b <= K0 || v.b <= kSuper) return false;
  const int M0 = K0 - K0 % kMega;
  const int Mend = v.b < M0 + kMega ? v.b : M0 + kMega;
  const int Kend = v.b < K0 + kSuper ? v.b : K0 + kSuper;
  if (Mend - M0 <= Kend - K0) return false;       // the mega-panel is this super-panel
  const int span = inv_span(v.b);
  GemmDesc g{};
  g.M = v.b; g.N = Mend - M0; g.K = kSuper;
  g.A = v.spanel; g.sA = (long long)v.b * span; g.lda = kSuper;
  g.B = (double2*)v.sbrow + M0; g.sB = (long long)span * v.b; g.ldb = v.b;
  g.C = (double2*)v.S + M0; g.sC = v.sS; g.ldc = v.b;
  g.D = (double2*)v.S + M0; g.sD = v.sS; g.ldd = v.b;
  g.alpha = zc{1.0, 0.0};
  g.beta = zc{1.0, 0.0};
  g.batch = v.batch; g.batch2 = 1;
  g.tiles = inv_update_tiles(g.M, g.N);
  *out = g;
  return true;
}
// The rank-kMega update after the mega-panel at M0: the columns left of it
// (side 0) or right of it (side 1); false when there are none or the matrix
// has a single mega-panel.
__host__ __device__ inline bool inv_mega_update(const InvDesc& v, int M0, int side,
                                                GemmDesc* out) {
  if (v.b <= kMega || v.b <= M0) return false;
  const int Mend = v.b < M0 + kMega ? v.b : M0 + kMega;
  const int c0 = side == 0 ? 0 : Mend;
  const int nc = side == 0 ? M0 : v.b - Mend;
  if (nc <= 0) return false;
  GemmDesc g{};
  g.M = v.b; g.N = nc; g.K = Mend - M0;
  g.A = v.spanel; g.sA = (long long)v.b * kMega; g.lda = kMega;
  g.B = (double2*)v.sbrow + c0; g.sB = (long long)kMega * v.b; g.ldb = v.b;
  g.C = (double2*)v.S + c0; g.sC = v.sS; g.ldc = v.b;
  g.D = (double2*)v.S + c0; g.sD = v.sS; g.ldd = v.b;
  g.alpha = zc{1.0, 0.0};
  g.beta = zc{1.0, 0.0};
  g.batch = v.batch; g.batch2 = 1;
  g.tiles = ((g.M + kMegaTile - 1) / kMegaTile) * ((g.N + kMegaTile - 1) / kMegaTile);
  *out = g;
  return true;
}

// Matrices of b <= kSmallB are inverted whole by one workgroup each, in one
// launch (registers hold the matrix: rpl = 1 for b <= 64, 2 for b <= 128;
// 256 rpl threads).  The result is written permuted to X; S is only read,
// and the work buffers are not used.
constexpr int kSmallB = 128;
inline int small_rpl(int b) { return b <= 64 ? 1 : 2; }
hipError_t launch_inv_small(int rpl, const FlatLaunch& l, hipStream_t s);

// Final permutation X[k][p_j] = S[p_k][j]; 8 rows per workgroup.
constexpr int kPermRows = 8;
hipError_t launch_inv_permute(const FlatLaunch& l, hipStream_t s);

// ---- elementwise ------------------------------------------------------------
// D[e] = idc(e) I + sum_t (c_t + d_t E[e]) Src_t[e]; idc(e) = idc0 + idc1 E[e].
struct LinCombDesc {
  const void* src[3];
  long long sSrc[3];
  zc c[3], d[3];
  zc idc0, idc1;
  void* D;
  long long sD;
  const double* E;     // device, [batch] (may be null if unused)
  int b;
  int batch;
};
constexpr int kLinChunk = 2048;      // elements per workgroup
// D[e] = a C[e] + z Z[e] + g Z[e]^dagger (32 x 32 tiles through LDS).
struct TransDesc {
  const void* C;
  const void* Z;
  void* D;
  long long sC, sZ, sD;
  zc a, z, g;
  int b;
  int batch;
};
constexpr int kTransTile = 32;
hipError_t launch_lincomb(const FlatLaunch& l, hipStream_t s);
hipError_t launch_transcomb(const FlatLaunch& l, hipStream_t s);
// Per energy: dos[n], density[n] from the diagonal blocks of G^< / G^>,
// current[n-1] from the lower blocks of G^< and Hd = H_{i,i+1}^dagger
// ([n-1][b][b], shared by all energies) through partial sums in `part`
// (observables_part_bytes).  Null outputs are skipped.
size_t observables_part_bytes(int n, int b, int batch);
hipError_t launch_observables(const void* gl_d, const void* gg_d, const void* gl_l,
                              const void* hd, double* dos, double* dens, double* cur, int n,
                              int b, int batch, double* part, hipStream_t s);
// B[k][i] = s * sum_{k'} X1'[k + shift - k'][i] X2[k'][i] (X1' = X1, or X1
// reversed in energy when rev), [energy][n_elem] complex128, terms outside
// [0, n1) left out (convolution.hip).
hipError_t launch_energy_convolution(const void* X1, int n1, int rev, const void* X2, int n2,
                                     void* B, int n_out, int shift, double s_re, double s_im,
                                     long long n_elem, hipStream_t st);
// L_e = -f_e (S_e - S_e^dagger), G_e = (1 - f_e)(S_e - S_e^dagger) with
// occ[2e] = f_e, occ[2e + 1] = 1 - f_e (device); S_e at stride sS (0 = shared),
// L and G contiguous, either may be null.
hipError_t launch_lesser_greater(const void* S, long long sS, const double* occ, void* L,
                                 void* G, int b, int batch, hipStream_t s);
// Per-matrix norms in two passes (partial sums per chunk, then per matrix);
// `part` is device scratch of norm_scratch_bytes(bb, batch) bytes.
constexpr long long kNormChunkElems = 8192;
inline int norm_chunks(long long bb) {
  const long long c = (bb + kNormChunkElems - 1) / kNormChunkElems;
  return (int)(c < 1 ? 1 : (c > 64 ? 64 : c));
}
inline size_t norm_scratch_bytes(long long bb, int batch) {
  return (size_t)batch * norm_chunks(bb) * 4 * sizeof(double) + 256;
}
// out[e] = ||x_e - prev_e||_F / ||x_e||_F for `batch` contiguous matrices of
// bb complex elements each.
hipError_t launch_update_norm(const void* x, const void* prev, double* out, long long bb,
                              int batch, double* part, hipStream_t s);
// out[e] = (||a_e||_F + ||c_e||_F) / (||a0_e||_F + ||c0_e||_F); a, c contiguous,
// a0, c0 at strides sa0, sc0 (0 = one shared block).
hipError_t launch_coupling_norm(const void* a, const void* c, const void* a0, long long sa0,
                                const void* c0, long long sc0, double* out, long long bb,
                                int batch, double* part, hipStream_t s);

// workgroups per matrix of the elementwise kernels
__host__ __device__ inline int lincomb_chunks(int b) { return (int)(((long long)b * b + kLinChunk - 1) / kLinChunk); }
__host__ __device__ inline int trans_tiles(int b) {
  const int t = (b + kTransTile - 1) / kTransTile;
  return t * t;
}

// Device-side binary search of the descriptor owning workgroup w.
__device__ __forceinline__ int find_desc(const int* prefix, int nd, int w) {
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= w) lo = mid; else hi = mid - 1;
  }
  return lo;
}

}  // namespace qtx
