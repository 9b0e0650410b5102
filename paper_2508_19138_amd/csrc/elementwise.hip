// Elementwise kernels over b x b complex128 blocks: system assembly
// (G-type  Mt = E S - H - Sigma^R, and the identity term of the W-type
// Mt = I - V P^R), anti-Hermitian-part updates (Z - Z^dagger) and adjoint
// copies (lower = -upper^dagger).  HBM-bound; rows are read and written
// contiguously, the adjoint goes through a 32 x 32 LDS tile.
#include "qtx_internal.h"

namespace qtx {
namespace {

__global__ __launch_bounds__(256)
void lincomb_kernel(FlatLaunch L) {
  const int di = find_desc(L.prefix, L.nd, blockIdx.x);
  const LinCombDesc& a = ((const LinCombDesc*)L.desc)[di];
  const int b = a.b;
  const int chunks = lincomb_chunks(b);
  const int local = blockIdx.x - L.prefix[di];
  const long long e = local / chunks;
  const long long q0 = (long long)(local % chunks) * kLinChunk;
  const long long nel = (long long)b * b;
  const double E = a.E ? a.E[e] : 0.0;
  zc co[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) co[t] = zc{a.c[t].re + a.d[t].re * E, a.c[t].im + a.d[t].im * E};
  const zc id = zc{a.idc0.re + a.idc1.re * E, a.idc0.im + a.idc1.im * E};
  double2* D = (double2*)a.D + e * a.sD;
  const double2* S0 = a.src[0] ? (const double2*)a.src[0] + e * a.sSrc[0] : nullptr;
  const double2* S1 = a.src[1] ? (const double2*)a.src[1] + e * a.sSrc[1] : nullptr;
  const double2* S2 = a.src[2] ? (const double2*)a.src[2] + e * a.sSrc[2] : nullptr;
  const long long q1 = q0 + kLinChunk < nel ? q0 + kLinChunk : nel;
  // each thread owns kLinChunk / 256 elements; all of a source's loads are
  // issued together (out-of-range slots read element 0 and are dropped)
  constexpr int kPer = kLinChunk / 256;
  static_assert(kLinChunk % 256 == 0, "chunk");
  double2 acc[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const long long q = q0 + threadIdx.x + (long long)k * 256;
    const int r = (int)(q / b), c = (int)(q % b);
    acc[k] = (q < q1 && r == c) ? make_double2(id.re, id.im) : make_double2(0.0, 0.0);
  }
  const double2* src[3] = {S0, S1, S2};
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    if (!src[t]) continue;                      // uniform
    double2 v[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const long long q = q0 + threadIdx.x + (long long)k * 256;
      v[k] = src[t][q < q1 ? q : 0];
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) acc[k] = cadd(acc[k], cscale(co[t], v[k]));
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const long long q = q0 + threadIdx.x + (long long)k * 256;
    if (q < q1) D[q] = acc[k];
  }
}

__global__ __launch_bounds__(256)
void transcomb_kernel(FlatLaunch L) {
  __shared__ double2 tile[kTransTile][kTransTile + 1];
  const int di = find_desc(L.prefix, L.nd, blockIdx.x);
  const TransDesc& t = ((const TransDesc*)L.desc)[di];
  const int b = t.b;
  const int tiles = trans_tiles(b);
  const int tilesC = (b + kTransTile - 1) / kTransTile;
  const int local = blockIdx.x - L.prefix[di];
  const long long e = local / tiles;
  const int tl = local % tiles;
  const int r0 = (tl / tilesC) * kTransTile;
  const int c0 = (tl % tilesC) * kTransTile;
  const double2* C = t.C ? (const double2*)t.C + e * t.sC : nullptr;
  const double2* Z = t.Z ? (const double2*)t.Z + e * t.sZ : nullptr;
  double2* D = (double2*)t.D + e * t.sD;
  const bool useT = (t.g.re != 0.0 || t.g.im != 0.0) && Z;
  const bool useZ = (t.z.re != 0.0 || t.z.im != 0.0) && Z;
  const bool useC = (t.a.re != 0.0 || t.a.im != 0.0) && C;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  constexpr int kRows = kTransTile / 8;
  // loads are issued unconditionally (out-of-range slots read element 0 and
  // are replaced or dropped) so that each thread's loads overlap
  if (useT) {
    // tile[i][j] = Z[c0 + i][r0 + j]
    double2 v[kRows];
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      const int zr = c0 + ty + 8 * k, zcol = r0 + tx;
      const bool ok = zr < b && zcol < b;
      v[k] = Z[ok ? (long long)zr * b + zcol : 0];
      if (!ok) v[k] = make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int k = 0; k < kRows; ++k) tile[ty + 8 * k][tx] = v[k];
    __syncthreads();
  }
  double2 acc[kRows];
  long long qs[kRows];
  bool oks[kRows];
#pragma unroll
  for (int k = 0; k < kRows; ++k) {
    const int r = r0 + ty + 8 * k, c = c0 + tx;
    oks[k] = r < b && c < b;
    qs[k] = oks[k] ? (long long)r * b + c : 0;
    acc[k] = make_double2(0.0, 0.0);
  }
  if (useC) {
    double2 v[kRows];
#pragma unroll
    for (int k = 0; k < kRows; ++k) v[k] = C[qs[k]];
#pragma unroll
    for (int k = 0; k < kRows; ++k) acc[k] = cscale(t.a, v[k]);
  }
  if (useZ) {
    double2 v[kRows];
#pragma unroll
    for (int k = 0; k < kRows; ++k) v[k] = Z[qs[k]];
#pragma unroll
    for (int k = 0; k < kRows; ++k) acc[k] = cadd(acc[k], cscale(t.z, v[k]));
  }
#pragma unroll
  for (int k = 0; k < kRows; ++k) {
    if (useT) acc[k] = cadd(acc[k], cscale(t.g, cconj(tile[tx][ty + 8 * k])));   // conj(Z[c][r])
    if (oks[k]) D[qs[k]] = acc[k];
  }
}

// Lesser/greater boundary blocks from the retarded one, both outputs in one
// pass: d = S - S^dagger per 32 x 32 tile (the transposed tile through LDS),
// then L = -f_e d and G = (1 - f_e) d.  Grid: batch x trans_tiles(b).
__global__ __launch_bounds__(256)
void lesser_greater_kernel(const double2* __restrict__ S, long long sS,
                           const double* __restrict__ occ, double2* __restrict__ L,
                           double2* __restrict__ G, int b) {
  __shared__ double2 tile[kTransTile][kTransTile + 1];
  const int tiles = trans_tiles(b);
  const int tilesC = (b + kTransTile - 1) / kTransTile;
  const long long e = blockIdx.x / tiles;
  const int tl = blockIdx.x % tiles;
  const int r0 = (tl / tilesC) * kTransTile;
  const int c0 = (tl % tilesC) * kTransTile;
  const long long bb = (long long)b * b;
  const double2* Se = S + e * sS;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  constexpr int kRows = kTransTile / 8;
  // tile[i][j] = S[c0 + i][r0 + j]; out-of-range slots read element 0
#pragma unroll
  for (int k = 0; k < kRows; ++k) {
    const int zr = c0 + ty + 8 * k, zc = r0 + tx;
    const bool ok = zr < b && zc < b;
    double2 v = Se[ok ? (long long)zr * b + zc : 0];
    if (!ok) v = make_double2(0.0, 0.0);
    tile[ty + 8 * k][tx] = v;
  }
  __syncthreads();
  const double f = occ[2 * e], g = occ[2 * e + 1];
#pragma unroll
  for (int k = 0; k < kRows; ++k) {
    const int r = r0 + ty + 8 * k, c = c0 + tx;
    if (r < b && c < b) {
      const double2 s = Se[(long long)r * b + c];
      const double2 t = tile[tx][ty + 8 * k];          // S[c][r]
      const double dx = s.x - t.x, dy = s.y + t.y;     // (S - S^dagger)[r][c]
      const long long q = e * bb + (long long)r * b + c;
      if (L) L[q] = make_double2(-f * dx, -f * dy);
      if (G) G[q] = make_double2(g * dx, g * dy);
    }
  }
}

// Sums of squared moduli over matrices, in two passes so that every matrix
// is spread over many workgroups: pass one writes per-chunk partial sums of
// up to four terms (|u|^2, or |u - v|^2 when v is given), pass two combines
// them per matrix.  Deterministic: fixed chunking and reduction order.
struct NormTerms {
  const double2* u[4];
  const double2* v[4];
  long long su[4], sv[4];
  int nt;
};

__global__ __launch_bounds__(256)
void norm_partial_kernel(NormTerms T, long long bb, int chunks, double* __restrict__ part) {
  const long long e = blockIdx.x / chunks;
  const int ch = blockIdx.x % chunks;
  const long long per = (bb + chunks - 1) / chunks;
  const long long q0 = ch * per;
  const long long q1 = q0 + per < bb ? q0 + per : bb;
  const int t = threadIdx.x;
  __shared__ double red[4][256];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double acc = 0.0;
    if (k < T.nt) {                          // uniform across the workgroup
      const double2* u = T.u[k] + e * T.su[k];
      const double2* v = T.v[k] ? T.v[k] + e * T.sv[k] : nullptr;
      for (long long q = q0 + t; q < q1; q += 256) {
        double2 a = u[q];
        if (v) {
          const double2 w = v[q];
          a.x -= w.x;
          a.y -= w.y;
        }
        acc += a.x * a.x + a.y * a.y;
      }
    }
    red[k][t] = acc;
  }
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) {
#pragma unroll
      for (int k = 0; k < 4; ++k) red[k][t] += red[k][t + h];
    }
    __syncthreads();
  }
  if (t < 4) part[(e * chunks + ch) * 4 + t] = red[t][0];
}

// mode 0: ||u0 - v0|| / ||u1|| (the relative update; infinite if ||u1|| = 0
// and the update is not); mode 1: (||u0|| + ||u1||) / (||u2|| + ||u3||)
__global__ __launch_bounds__(256)
void norm_final_kernel(const double* __restrict__ part, int chunks, int batch, int mode,
                       double* __restrict__ out) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= batch) return;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int ch = 0; ch < chunks; ++ch)
#pragma unroll
    for (int k = 0; k < 4; ++k) s[k] += part[((long long)e * chunks + ch) * 4 + k];
  if (mode == 0) {
    out[e] = s[1] > 0.0 ? sqrt(s[0]) / sqrt(s[1]) : (s[0] > 0.0 ? HUGE_VAL : 0.0);
  } else {
    const double num = sqrt(s[0]) + sqrt(s[1]);
    const double den = sqrt(s[2]) + sqrt(s[3]);
    out[e] = den > 0.0 ? num / den : 0.0;
  }
}

hipError_t launch_norms(const NormTerms& T, long long bb, int batch, int mode, double* out,
                        double* part, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  const int chunks = norm_chunks(bb);
  hipLaunchKernelGGL(norm_partial_kernel, dim3((unsigned)((long long)batch * chunks)), dim3(256),
                     0, s, T, bb, chunks, part);
  hipLaunchKernelGGL(norm_final_kernel, dim3((batch + 255) / 256), dim3(256), 0, s, part, chunks,
                     batch, mode, out);
  return hipGetLastError();
}

// The current through interface i, 2 Re Tr(H_{i,i+1} G^<_{i+1,i}) =
// 2 sum_q Re(G[q] conj(Hd[q])) with Hd = H_{i,i+1}^dagger (both blocks read
// contiguously), in partial sums: workgroup (i, tile) keeps its tile of Hd
// in registers and streams the same tile of G^<_{i+1,i} of every energy,
// kObsEnergies energies per pass, so each coupling block is read once per
// call rather than once per energy.  part[(e (n-1) + i) tiles + tile].
constexpr int kObsVec = 8;                      // elements per thread and tile
constexpr int kObsTile = 256 * kObsVec;         // elements per workgroup
constexpr int kObsEnergies = 8;                 // energies per pass

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) x += __shfl_xor(x, m, 64);
  return x;
}

__global__ __launch_bounds__(256)
void current_partial_kernel(const double2* __restrict__ gl_l, const double2* __restrict__ hd,
                            double* __restrict__ part, int n, int b, int batch, int tiles) {
  const int i = blockIdx.x / tiles, tl = blockIdx.x % tiles;
  const long long bb = (long long)b * b;
  const long long q0 = (long long)tl * kObsTile;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  double2 h[kObsVec];
#pragma unroll
  for (int v = 0; v < kObsVec; ++v) {
    const long long q = q0 + t + 256 * v;
    h[v] = q < bb ? hd[(long long)i * bb + q] : make_double2(0.0, 0.0);
  }
  __shared__ double red[kObsEnergies][4];
  for (int e0 = 0; e0 < batch; e0 += kObsEnergies) {
    double sum[kObsEnergies];
#pragma unroll
    for (int k = 0; k < kObsEnergies; ++k) {
      sum[k] = 0.0;
      const int e = e0 + k;
      if (e < batch) {                          // uniform across the workgroup
        const double2* G = gl_l + ((long long)e * (n - 1) + i) * bb;
#pragma unroll
        for (int v = 0; v < kObsVec; ++v) {
          const long long q = q0 + t + 256 * v;
          if (q < bb) {
            const double2 g = G[q];
            sum[k] = fma(g.x, h[v].x, fma(g.y, h[v].y, sum[k]));
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kObsEnergies; ++k) {
      const double w = wave_sum(sum[k]);
      if (lane == 0) red[k][wave] = w;
    }
    __syncthreads();
    if (t < kObsEnergies && e0 + t < batch)
      part[((long long)(e0 + t) * (n - 1) + i) * tiles + tl] =
          (red[t][0] + red[t][1]) + (red[t][2] + red[t][3]);
    __syncthreads();
  }
}

// Observables per energy e: workgroups k < n take block k's traces
// (density of states from i(G^> - G^<), density from -i G^<, diagonal
// elements only), workgroups k >= n the current through interface
// i = k - n from its partial sums.
__global__ __launch_bounds__(256)
void observables_kernel(const double2* __restrict__ gl_d, const double2* __restrict__ gg_d,
                        const double* __restrict__ part, int tiles,
                        double* __restrict__ dos, double* __restrict__ dens,
                        double* __restrict__ cur, int n, int b) {
  const int per = 2 * n - 1;
  const long long e = blockIdx.x / per;
  const int k = blockIdx.x % per;
  const long long bb = (long long)b * b;
  const int t = threadIdx.x;
  double s0 = 0.0, s1 = 0.0;
  if (k < n) {
    // gg_d is null when no density of states is asked for (uniform branch)
    const double2* L = gl_d + (e * n + k) * bb;
    const double2* Gg = gg_d ? gg_d + (e * n + k) * bb : nullptr;
    for (int j = t; j < b; j += 256) {
      const double2 l = L[(long long)j * (b + 1)];
      const double2 g = Gg ? Gg[(long long)j * (b + 1)] : make_double2(0.0, 0.0);
      s0 += l.y - g.y;          // Re(i (g - l))
      s1 += l.y;                // Re(-i l)
    }
  } else if (cur) {             // part is null when no current is asked for
    const int i = k - n;
    const double* P = part + (e * (n - 1) + i) * tiles;
    for (int q = t; q < tiles; q += 256) s0 += P[q];
  }
  __shared__ double r0[256], r1[256];
  r0[t] = s0;
  r1[t] = s1;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) {
      r0[t] += r0[t + h];
      r1[t] += r1[t + h];
    }
    __syncthreads();
  }
  if (t == 0) {
    const double inv2pi = 0.15915494309189533577;   // 1 / (2 pi)
    if (k < n) {
      if (dos) dos[e * n + k] = r0[0] * inv2pi;
      if (dens) dens[e * n + k] = r1[0] * inv2pi;
    } else if (cur) {
      cur[e * (n - 1) + (k - n)] = 2.0 * r0[0] * inv2pi;
    }
  }
}

}  // namespace

size_t observables_part_bytes(int n, int b, int batch) {
  if (n < 2) return 0;
  const long long tiles = ((long long)b * b + kObsTile - 1) / kObsTile;
  return (size_t)batch * (n - 1) * tiles * sizeof(double);
}

hipError_t launch_observables(const void* gl_d, const void* gg_d, const void* gl_l,
                              const void* hd, double* dos, double* dens, double* cur, int n,
                              int b, int batch, double* part, hipStream_t s) {
  if (batch <= 0 || n <= 0) return hipSuccess;
  const int tiles = (int)(((long long)b * b + kObsTile - 1) / kObsTile);
  if (cur && n > 1) {
    hipLaunchKernelGGL(current_partial_kernel, dim3((unsigned)((n - 1) * tiles)), dim3(256), 0,
                       s, (const double2*)gl_l, (const double2*)hd, part, n, b, batch, tiles);
  }
  const long long grid = (long long)batch * (2 * n - 1);
  hipLaunchKernelGGL(observables_kernel, dim3((unsigned)grid), dim3(256), 0, s,
                     (const double2*)gl_d, (const double2*)gg_d,
                     (cur && n > 1) ? (const double*)part : nullptr, tiles, dos, dens,
                     (cur && n > 1) ? cur : nullptr, n, b);
  return hipGetLastError();
}

hipError_t launch_lesser_greater(const void* S, long long sS, const double* occ, void* L,
                                 void* G, int b, int batch, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  const long long grid = (long long)batch * trans_tiles(b);
  hipLaunchKernelGGL(lesser_greater_kernel, dim3((unsigned)grid), dim3(256), 0, s,
                     (const double2*)S, sS, occ, (double2*)L, (double2*)G, b);
  return hipGetLastError();
}

hipError_t launch_coupling_norm(const void* a, const void* c, const void* a0, long long sa0,
                                const void* c0, long long sc0, double* out, long long bb,
                                int batch, double* part, hipStream_t s) {
  NormTerms T{};
  T.u[0] = (const double2*)a;  T.su[0] = bb;
  T.u[1] = (const double2*)c;  T.su[1] = bb;
  T.u[2] = (const double2*)a0; T.su[2] = sa0;
  T.u[3] = (const double2*)c0; T.su[3] = sc0;
  T.nt = 4;
  return launch_norms(T, bb, batch, 1, out, part, s);
}

hipError_t launch_update_norm(const void* x, const void* prev, double* out, long long bb,
                              int batch, double* part, hipStream_t s) {
  NormTerms T{};
  T.u[0] = (const double2*)x; T.v[0] = (const double2*)prev; T.su[0] = bb; T.sv[0] = bb;
  T.u[1] = (const double2*)x; T.su[1] = bb;
  T.nt = 2;
  return launch_norms(T, bb, batch, 0, out, part, s);
}

hipError_t launch_lincomb(const FlatLaunch& l, hipStream_t s) {
  if (l.total <= 0) return hipSuccess;
  hipLaunchKernelGGL(lincomb_kernel, dim3(l.total), dim3(256), 0, s, l);
  return hipGetLastError();
}

hipError_t launch_transcomb(const FlatLaunch& l, hipStream_t s) {
  if (l.total <= 0) return hipSuccess;
  hipLaunchKernelGGL(transcomb_kernel, dim3(l.total), dim3(256), 0, s, l);
  return hipGetLastError();
}

}  // namespace qtx
