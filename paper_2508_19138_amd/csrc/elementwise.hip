// Elementwise kernels over b x b complex128 blocks: system assembly
// (G-type  Mt = E S - H - Sigma^R, and the identity term of the W-type
// Mt = I - V P^R), anti-Hermitian-part updates (Z - Z^dagger) and adjoint
// copies (lower = -upper^dagger).  All HBM-bound; coalesced along rows.
#include "qtx_internal.h"

namespace qtx {
namespace {

__global__ __launch_bounds__(256)
void lincomb_kernel(int b, LinComb a) {
  const long long e = blockIdx.y;
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
  for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < nel;
       q += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(q / b), c = (int)(q % b);
    double2 v = (r == c) ? make_double2(id.re, id.im) : make_double2(0.0, 0.0);
    if (S0) v = cadd(v, cscale(co[0], S0[q]));
    if (S1) v = cadd(v, cscale(co[1], S1[q]));
    if (S2) v = cadd(v, cscale(co[2], S2[q]));
    D[q] = v;
  }
}

// 32 x 32 tiles; the transposed operand goes through LDS.
constexpr int kTT = 32;

__global__ __launch_bounds__(256)
void transcomb_kernel(int b, TransComb t) {
  __shared__ double2 tile[kTT][kTT + 1];
  const long long e = blockIdx.z;
  const int tilesC = (b + kTT - 1) / kTT;
  const int r0 = (blockIdx.x / tilesC) * kTT;
  const int c0 = (blockIdx.x % tilesC) * kTT;
  const double2* C = t.C ? (const double2*)t.C + e * t.sC : nullptr;
  const double2* Z = t.Z ? (const double2*)t.Z + e * t.sZ : nullptr;
  double2* D = (double2*)t.D + e * t.sD;
  const bool useT = (t.g.re != 0.0 || t.g.im != 0.0) && Z;
  const bool useZ = (t.z.re != 0.0 || t.z.im != 0.0) && Z;
  const bool useC = (t.a.re != 0.0 || t.a.im != 0.0) && C;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  if (useT) {
    // tile[i][j] = Z[c0 + i][r0 + j]  (rows of Z^dagger's source)
    for (int i = ty; i < kTT; i += 8) {
      const int zr = c0 + i, zc_ = r0 + tx;
      tile[i][tx] = (zr < b && zc_ < b) ? Z[(long long)zr * b + zc_] : make_double2(0.0, 0.0);
    }
    __syncthreads();
  }
  for (int i = ty; i < kTT; i += 8) {
    const int r = r0 + i, c = c0 + tx;
    if (r >= b || c >= b) continue;
    const long long q = (long long)r * b + c;
    double2 v = make_double2(0.0, 0.0);
    if (useC) v = cscale(t.a, C[q]);
    if (useZ) v = cadd(v, cscale(t.z, Z[q]));
    if (useT) v = cadd(v, cscale(t.g, cconj(tile[tx][i])));   // conj(Z[c][r])
    D[q] = v;
  }
}

__global__ __launch_bounds__(256)
void nonfinite_kernel(const double2* __restrict__ p, long long count, int* flag) {
  int bad = 0;
  for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < count;
       q += (long long)gridDim.x * blockDim.x) {
    const double2 v = p[q];
    if (!(fabs(v.x) <= 1.7976931348623157e308) || !(fabs(v.y) <= 1.7976931348623157e308)) bad = 1;
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

}  // namespace

hipError_t launch_lincomb(int b, int batch, const LinComb& a, hipStream_t s) {
  if (batch <= 0 || b <= 0) return hipSuccess;
  const long long nel = (long long)b * b;
  int blocks = (int)((nel + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(lincomb_kernel, dim3(blocks, batch), dim3(256), 0, s, b, a);
  return hipGetLastError();
}

hipError_t launch_transcomb(int b, int batch, const TransComb& t, hipStream_t s) {
  if (batch <= 0 || b <= 0) return hipSuccess;
  const int tiles = (b + kTT - 1) / kTT;
  hipLaunchKernelGGL(transcomb_kernel, dim3(tiles * tiles, 1, batch), dim3(256), 0, s, b, t);
  return hipGetLastError();
}

hipError_t launch_nonfinite_scan(const void* p, long long count, int* flag,
                                 hipStream_t s) {
  if (count <= 0) return hipSuccess;
  long long blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(nonfinite_kernel, dim3((int)blocks), dim3(256), 0, s,
                     (const double2*)p, count, flag);
  return hipGetLastError();
}

}  // namespace qtx
