// Host-side internal interfaces of the RGF library: kernel launchers and
// the argument blocks they take.  Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qtx_device.h"

namespace qtx {

constexpr int kMaxGroups = 4;

// One independent strided-batched product inside a grouped launch:
//   D[e] = alpha * op(A[e]) op(B[e]) + beta * C[e]
// Element e of an operand starts at ptr + e * stride (stride 0 = shared).
struct GemmGroup {
  const void* A;
  const void* B;
  const void* C;
  void* D;
  long long sA, sB, sC, sD;   // strides over the first batch index (energy)
  long long tA, tB, tC, tD;   // strides over the second batch index (block)
  zc alpha, beta;
};

// Up to kMaxGroups products sharing the shape, the operations and the
// leading dimensions are issued as one launch.
struct GemmArgs {
  int M, N, K;
  long long lda, ldb, ldc, ldd;
  int batch;        // first batch index  (grid y = batch * batch2)
  int batch2;       // second batch index (0 is read as 1)
  int ngroups;
  GemmGroup g[kMaxGroups];
};

// opa/opb: 'N' or 'C'.  FP64: complex128 operands on the FP64 matrix cores.
hipError_t launch_zgemm(char opa, char opb, const GemmArgs& a, hipStream_t s);
// FP32: complex64 operands on the FP32 matrix cores (alpha/beta rounded).
hipError_t launch_cgemm(char opa, char opb, const GemmArgs& a, hipStream_t s);

// ---- Gauss-Jordan inverse with partial pivoting --------------------------
constexpr int kPanel = 16;   // panel width (columns per factorisation step)

struct InvWork {
  void* panel;      // [batch][b][kPanel] complex128
  void* brow;       // [batch][kPanel][b] complex128
  int* perm;        // [batch][b]
  int* used;        // [batch][b]
};
// In-place GJ on S[e] (stride sS, b x b); result, un-permuted, into X[e].
// info[e] (may be null): 0 if fine, else set once to +code (zero pivot) or
// -code (non-finite pivot); code = 1 + column when code_base <= 0, else
// code_base.
hipError_t launch_zinv(int b, void* S, long long sS, void* X, long long sX,
                       int batch, const InvWork& w, int* info, int code_base,
                       hipStream_t s);

// ---- elementwise kernels -------------------------------------------------
// D[e] = idc(e) * I + sum_t (c_t + d_t * E[e]) * Src_t[e] over b x b blocks,
// idc(e) = idc0 + idc1 * E[e].  Null sources are skipped; E may be null when
// every d_t and idc1 is zero.
struct LinComb {
  const void* src[3];
  long long sSrc[3];
  zc c[3], d[3];
  zc idc0, idc1;
  void* D;
  long long sD;
  const double* E;   // device array, [batch]
};
hipError_t launch_lincomb(int b, int batch, const LinComb& a, hipStream_t s);

// D[e] = a * C[e] + z * Z[e] + g * Z[e]^dagger  (C or Z may be null when its
// coefficient is zero; C may equal D; Z must not alias D unless g == 0).
struct TransComb {
  const void* C;
  const void* Z;
  void* D;
  long long sC, sZ, sD;
  zc a, z, g;
};
hipError_t launch_transcomb(int b, int batch, const TransComb& t, hipStream_t s);

// Count of non-finite entries over `count` complex128 values (device),
// accumulated into *flag (device int).
hipError_t launch_nonfinite_scan(const void* p, long long count, int* flag,
                                 hipStream_t s);

}  // namespace qtx
