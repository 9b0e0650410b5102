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
// the per-matrix status words are cleared by the first panel kernel (or by
// the one-workgroup inverse, for b <= kSmallB).
#include <mutex>
#include <string>

#include "../../include/qtx_rgf.h"
#include "ctx.h"
#include "exec.h"

namespace qtx {
namespace {

constexpr size_t kScratchBytes = (size_t)QTX_NOALLOC_SCRATCH_BYTES;
// descriptor tables: one InvDesc, the update products' descriptors, and
// the prefix arrays of every launch
constexpr size_t kDescBytes = 64 << 10;
constexpr int kMaxUpdates = 1024 / kPanel + 1024 / kSuper + 2 * (1024 / kMega);
constexpr int kMaxSteps = 2 * (1024 / kPanel) + 2 * (1024 / kSuper) + 2 * (1024 / kMega) + 1;

static __device__ __align__(256) char scratch[kScratchBytes + kDescBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_ptr[kMaxDevices] = {};

// One launch of the inverse: a panel at k0, a gather of the W-column panel
// at k0, `count` update products from upd[first] (tile configuration cfg),
// or the final permutation.
struct Step {
  int kind;                  // 0 panel, 1 products, 2 gather, 3 permutation, 4 whole (b <= kSmallB)
  int k0, W, cfg;
  int first, count;
};

// Layout of the descriptor area.
struct DescArea {
  InvDesc inv;
  GemmDesc upd[kMaxUpdates];
  Step steps[kMaxSteps];
  int pre[kMaxSteps][3];     // prefix array of every launch
};
static_assert(sizeof(DescArea) <= kDescBytes, "descriptor area");

// The executor's launch sequence for one inverse operation, in order: for
// b <= kSmallB the one-workgroup inverse alone; else per mega-panel, per
// super-panel, each panel and its rank-kPanel update, then the
// super-panel's gather and rank-kSuper update of the mega-panel's columns;
// after the mega-panel its gather and rank-kMega update of the other
// columns; the permutation last.  Returns the number of steps.
__host__ __device__ inline int inv_steps(const InvDesc& v, Step* st, GemmDesc* upd) {
  int ns = 0, nu = 0;
  if (v.b <= kSmallB) {
    st[ns++] = Step{4, 0, 0, 0, 0, 0};
    return ns;
  }
  for (int M0 = 0; M0 < v.b; M0 += kMega) {
    const int mend = v.b < M0 + kMega ? v.b : M0 + kMega;
    for (int K0 = M0; K0 < mend; K0 += kSuper) {
      const int kend = v.b < K0 + kSuper ? v.b : K0 + kSuper;
      for (int k0 = K0; k0 < kend; k0 += kPanel) {
        st[ns++] = Step{0, k0, 0, 0, 0, 0};
        if (inv_panel_update(v, k0, &upd[nu])) {
          st[ns++] = Step{1, k0, 0, kGemmInvUpdate, nu, 1};
          ++nu;
        }
      }
      if (inv_super_update(v, K0, &upd[nu])) {
        st[ns++] = Step{2, K0, kSuper, 0, 0, 0};
        st[ns++] = Step{1, K0, 0, kGemmInvUpdate, nu, 1};
        ++nu;
      }
    }
    int c = 0;
    for (int side = 0; side < 2; ++side)
      if (inv_mega_update(v, M0, side, &upd[nu + c])) ++c;
    if (c) {
      st[ns++] = Step{2, M0, kMega, 0, 0, 0};
      st[ns++] = Step{1, M0, 0, kMegaCfg, nu, c};
      nu += c;
    }
  }
  st[ns++] = Step{3, 0, 0, 0, 0, 0};
  return ns;
}

// workgroups of a step
__host__ __device__ inline int step_total(const InvDesc& v, const Step& t, const GemmDesc* upd) {
  switch (t.kind) {
    case 0:
    case 4: return v.batch;
    case 2: return v.batch * super_gather_chunks(v.b, t.W);
    case 3: return v.batch * ((v.b + kPermRows - 1) / kPermRows);
    default: {
      int n = 0;
      for (int q = 0; q < t.count; ++q) n += upd[t.first + q].tiles * upd[t.first + q].batch;
      return n;
    }
  }
}

__global__ void noalloc_setup_kernel(InvDesc v, DescArea* a) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  a->inv = v;
  Step* st = a->steps;       // in the descriptor area: no private stack array
  const int ns = inv_steps(v, st, a->upd);
  for (int i = 0; i < ns; ++i) {
    a->pre[i][0] = 0;
    if (st[i].kind == 1) {
      for (int q = 0; q < st[i].count; ++q) {
        const GemmDesc& g = a->upd[st[i].first + q];
        a->pre[i][q + 1] = a->pre[i][q] + g.tiles * g.batch;
      }
    } else {
      a->pre[i][1] = step_total(v, st[i], a->upd);
    }
  }
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

size_t noalloc_work_bytes(int b, int batch) {
  if (b <= kSmallB) return 0;          // the one-launch inverse uses no work buffers
  const size_t pan = align256((size_t)batch * b * kPanel * 16);
  const size_t span = align256((size_t)batch * b * inv_span(b) * 16);
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
  const size_t span = align256((size_t)batch * b * inv_span(b) * 16);
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
  Step st[kMaxSteps];
  const int n_steps = inv_steps(v, st, upd);
  const hipStream_t s = c->stream;
  auto fail = [&](hipError_t e, const char* what) {
    c->err = std::string("qtx_rgf_zinv_noalloc: ") + what + ": " + hipGetErrorString(e);
    return QTX_ERR_HIP;
  };
  hipLaunchKernelGGL(noalloc_setup_kernel, dim3(1), dim3(64), 0, s, v, dev);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(e, "set-up launch");
  const int R = (b + kInvThreads - 1) / kInvThreads;
  for (int i = 0; i < n_steps; ++i) {
    const Step& t = st[i];
    const int total = step_total(v, t, upd);
    if (t.kind == 1) {
      const FlatLaunch l{&dev->upd[t.first], dev->pre[i], t.count, total};
      e = launch_gemm(t.cfg, false, 'N', 'N', l, s);
    } else {
      const FlatLaunch l{&dev->inv, dev->pre[i], 1, total};
      if (t.kind == 0) e = launch_inv_panel(R, t.k0, l, s);
      else if (t.kind == 4) e = launch_inv_small(small_rpl(b), l, s);
      else if (t.kind == 2) e = launch_inv_super_gather(t.k0, t.W, l, s);
      else e = launch_inv_permute(l, s);
    }
    if (e != hipSuccess) return fail(e, "launch");
  }
  // asynchronous: no wait, so the call can be captured into a graph
  return QTX_OK;
}
