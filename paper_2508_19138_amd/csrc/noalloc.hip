// The allocation-free variant of the batched inverse (qtx_rgf_zinv_noalloc)
// for callers that cannot allocate device memory: code under stream
// capture, tight serving loops.
//
// Its work buffers (panel, pivot rows, super-panel, permutation, used
// flags) and the descriptor tables of its launches live in one file-scope
// device array.  Every GPU the library runs on holds its own copy of the
// array, at its own address, until the process ends; the host learns that
// address once per device through hipGetSymbolAddress (at context
// creation) and only ever passes that address to kernels.  The descriptor
// tables are written on the device by a set-up kernel, so a call is a
// sequence of kernel launches on the context's stream and nothing else: no
// allocation, no copy, no memset, no wait.
//
// Calls on one GPU share the array: two calls that overlap in time on that
// GPU (different streams or contexts) race on it.  Nothing in the array
// needs to start at zero: every buffer is written before it is read, and
// the per-matrix status words are cleared by the first panel kernel.
#include <mutex>
#include <string>

#include "../../include/qtx_rgf.h"
#include "ctx.h"
#include "exec.h"

namespace qtx {
namespace {

constexpr size_t kScratchBytes = (size_t)QTX_NOALLOC_SCRATCH_BYTES;
// descriptor tables: one InvDesc, one GemmDesc per update product, and the
// prefix pairs of every launch
constexpr size_t kDescBytes = 64 << 10;
constexpr int kMaxUpdates = 1024 / kPanel + 1024 / kSuper;

static __device__ __align__(256) char scratch[kScratchBytes + kDescBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_ptr[kMaxDevices] = {};

// Layout of the descriptor area.
struct DescArea {
  InvDesc inv;
  GemmDesc upd[kMaxUpdates];
  int inv_pre[2];            // panel launches: one workgroup per matrix
  int gather_pre[2];
  int perm_pre[2];
  int upd_pre[kMaxUpdates][2];
};
static_assert(sizeof(DescArea) <= kDescBytes, "descriptor area");

// Update products in launch order: per super-panel, the rank-kPanel update
// after each panel that has one, then the rank-kSuper update.
__host__ __device__ inline int update_list(const InvDesc& v, GemmDesc* out) {
  int n = 0;
  for (int K0 = 0; K0 < v.b; K0 += kSuper) {
    const int end = v.b < K0 + kSuper ? v.b : K0 + kSuper;
    for (int k0 = K0; k0 < end; k0 += kPanel) {
      GemmDesc g;
      if (inv_panel_update(v, k0, &g)) { if (out) out[n] = g; ++n; }
    }
    GemmDesc g;
    if (inv_super_update(v, K0, &g)) { if (out) out[n] = g; ++n; }
  }
  return n;
}

__global__ void noalloc_setup_kernel(InvDesc v, DescArea* a) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  a->inv = v;
  const int n = update_list(v, a->upd);
  for (int i = 0; i < n; ++i) {
    a->upd_pre[i][0] = 0;
    a->upd_pre[i][1] = a->upd[i].tiles * a->upd[i].batch;
  }
  a->inv_pre[0] = 0;
  a->inv_pre[1] = v.batch;
  a->gather_pre[0] = 0;
  a->gather_pre[1] = v.batch * super_gather_chunks(v.b);
  a->perm_pre[0] = 0;
  a->perm_pre[1] = v.batch * ((v.b + kPermRows - 1) / kPermRows);
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

size_t noalloc_work_bytes(int b, int batch) {
  const size_t pan = align256((size_t)batch * b * kPanel * 16);
  const size_t span = align256((size_t)batch * b * kSuper * 16);
  const size_t ints = align256((size_t)batch * b * 4);
  return 2 * pan + 2 * span + 2 * ints;
}

hipError_t noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_mu);
  if (g_ptr[device]) return hipSuccess;
  // the caller has made `device` current
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_ptr[device] = (char*)p;
  return hipSuccess;
}

}  // namespace qtx

using namespace qtx;

extern "C" qtx_status qtx_rgf_zinv_noalloc(qtx_rgf_ctx* c, int32_t b, void* A, void* X,
                                           int32_t* info, int32_t batch) {
  if (!c || b < 1 || b > 1024 || !A || !X || batch < 0 || A == X) return QTX_ERR_INVALID_ARG;
  if (c->busy) return QTX_ERR_BUSY;
  c->err.clear();
  if (batch == 0) return QTX_OK;
  if (noalloc_work_bytes(b, batch) > kScratchBytes) {
    c->err = "qtx_rgf_zinv_noalloc: " + std::to_string(batch) + " matrices of size " +
             std::to_string(b) + " need " + std::to_string(noalloc_work_bytes(b, batch)) +
             " scratch bytes; the static scratch holds " + std::to_string(kScratchBytes);
    return QTX_ERR_INVALID_ARG;
  }
  char* base = nullptr;
  {
    std::lock_guard<std::mutex> g(g_mu);
    base = (c->device >= 0 && c->device < kMaxDevices) ? g_ptr[c->device] : nullptr;
  }
  if (!base) {
    c->err = "qtx_rgf_zinv_noalloc: the scratch address of this device is unknown";
    return QTX_ERR_HIP;
  }
  if (hipSetDevice(c->device) != hipSuccess) {
    (void)hipGetLastError();
    c->err = "hipSetDevice failed";
    return QTX_ERR_HIP;
  }
  const size_t pan = align256((size_t)batch * b * kPanel * 16);
  const size_t span = align256((size_t)batch * b * kSuper * 16);
  const size_t ints = align256((size_t)batch * b * 4);
  InvDesc v{};
  v.S = A; v.sS = (long long)b * b;
  v.X = X; v.sX = (long long)b * b;
  v.panel = base;
  v.brow = base + pan;
  v.spanel = base + 2 * pan;
  v.sbrow = base + 2 * pan + span;
  v.perm = (int*)(base + 2 * pan + 2 * span);
  v.used = (int*)(base + 2 * pan + 2 * span + ints);
  v.info = info; v.code = 0; v.reset_info = 1;
  v.b = b; v.batch = batch;
  DescArea* dev = (DescArea*)(base + kScratchBytes);

  // the same launch sequence as the executor's for one inverse operation
  GemmDesc upd[kMaxUpdates];
  const int n_upd = update_list(v, upd);
  const hipStream_t s = c->stream;
  auto fail = [&](hipError_t e, const char* what) {
    c->err = std::string("qtx_rgf_zinv_noalloc: ") + what + ": " + hipGetErrorString(e);
    return QTX_ERR_HIP;
  };
  hipLaunchKernelGGL(noalloc_setup_kernel, dim3(1), dim3(64), 0, s, v, dev);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(e, "set-up launch");
  const FlatLaunch inv_l{&dev->inv, dev->inv_pre, 1, batch};
  const int R = (b + kInvThreads - 1) / kInvThreads;
  int u = 0;
  for (int K0 = 0; K0 < b; K0 += kSuper) {
    const int end = std::min(b, K0 + kSuper);
    for (int k0 = K0; k0 < end; k0 += kPanel) {
      if ((e = launch_inv_panel(R, k0, inv_l, s)) != hipSuccess) return fail(e, "panel");
      GemmDesc g;
      if (inv_panel_update(v, k0, &g)) {
        const FlatLaunch l{&dev->upd[u], dev->upd_pre[u], 1, upd[u].tiles * batch};
        if ((e = launch_gemm(kGemmInvUpdate, false, 'N', 'N', l, s)) != hipSuccess)
          return fail(e, "panel update");
        ++u;
      }
    }
    GemmDesc g;
    if (inv_super_update(v, K0, &g)) {
      const FlatLaunch gl{&dev->inv, dev->gather_pre, 1, batch * super_gather_chunks(b)};
      if ((e = launch_inv_super_gather(K0, gl, s)) != hipSuccess) return fail(e, "gather");
      const FlatLaunch l{&dev->upd[u], dev->upd_pre[u], 1, upd[u].tiles * batch};
      if ((e = launch_gemm(kGemmInvUpdate, false, 'N', 'N', l, s)) != hipSuccess)
        return fail(e, "super-panel update");
      ++u;
    }
  }
  if (u != n_upd) {
    c->err = "qtx_rgf_zinv_noalloc: update count mismatch";
    return QTX_ERR_HIP;
  }
  const FlatLaunch pl{&dev->inv, dev->perm_pre, 1, batch * ((b + kPermRows - 1) / kPermRows)};
  if ((e = launch_inv_permute(pl, s)) != hipSuccess) return fail(e, "permute");
  // asynchronous: no wait, so the call can be captured into a graph
  return QTX_OK;
}
