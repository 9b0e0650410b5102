// C ABI of the RGF library: argument validation, lanes, admission of lanes
// into the workspace by footprint, and the merged execution of a batch.
//
// A batch of problems becomes a set of lanes (one problem, a contiguous
// chunk of its energies, its own workspace region).  Lanes are admitted into
// the workspace first-fit as memory frees up, and every admitted lane
// advances in the same merged launches (see exec.cpp), so solves of
// different block size, block count and kind share the GPU.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/qtx_rgf.h"
#include "ctx.h"
#include "emit.h"
#include "exec.h"

using namespace qtx;

namespace {

constexpr int kSplitMinEnergies = 64;          // energies before a problem is split
// Lanes of at most this many energies (independent single-energy solves)
// are spread over the pool's streams within their class: a class of many
// such lanes is a chain of latency-bound launches (one matrix per
// workgroup in the inverse's panels), and several shorter chains on
// different streams overlap one another's gaps.
constexpr int kSpreadMaxEnergies = 4;

}  // namespace

size_t qtx::budget_now(qtx_rgf_ctx* c) {
  if (c->budget) return c->budget;
  size_t fr = 0, tot = 0;
  HIPCHK(c, hipMemGetInfo(&fr, &tot));
  return (size_t)(0.9 * (double)(fr + c->ws_bytes));
}

void qtx::ensure(qtx_rgf_ctx* c, char** p, size_t* have, size_t need) {
  if (*have >= need) return;
  c->pool->sync();
  if (*p) {
    c->pool->release();             // cached graphs refer to the old memory
    (void)hipFree(*p);
    *p = nullptr;
    *have = 0;
  }
  if (hipMalloc((void**)p, need) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    c->err = "device allocation of " + std::to_string(need) + " bytes failed";
    throw Fail{QTX_ERR_NOMEM};
  }
  *have = need;
}

std::string qtx::validate_problem(const qtx_rgf_problem& p) {
  if (p.kind != QTX_KIND_G && p.kind != QTX_KIND_W) return "unknown kind";
  if (p.precision != QTX_FP64 && p.precision != QTX_MIXED) return "unknown precision";
  if (p.n_blocks < 1 || p.block_size < 1 || p.n_energies < 1)
    return "n_blocks, block_size and n_energies must be >= 1";
  if (p.block_size > kMaxB) return "block_size above 4096 is not supported";
  if (p.flags != 0) return "flags must be 0";
  if (!p.XR.diag) return "XR.diag is required";
  if (p.n_blocks > 1 && (!p.XR.upper || !p.XR.lower))
    return "XR.upper and XR.lower are required when n_blocks > 1";
  if (p.XL.diag && p.n_blocks > 1 && !p.XL.upper) return "XL.upper is required with XL.diag when n_blocks > 1";
  if (p.XG.diag && p.n_blocks > 1 && !p.XG.upper) return "XG.upper is required with XG.diag when n_blocks > 1";
  if (p.kind == QTX_KIND_G) {
    if (!p.energies) return "energies (host) are required for G-type problems";
    if (!p.H.diag || (p.n_blocks > 1 && !p.H.upper)) return "H.diag and H.upper are required";
    if (!p.sigma_r.diag) return "sigma_r.diag is required";
    if (!p.S.diag && (p.S.upper || p.S.lower)) return "S.upper/S.lower given without S.diag";
    if (p.XL.diag && !p.sigma_l.diag) return "sigma_l.diag is required for XL";
    if (p.XG.diag && !p.sigma_g.diag) return "sigma_g.diag is required for XG";
    if (p.WR_diag) return "WR_diag applies to W-type problems only";
  } else {
    if (!p.V.diag || (p.n_blocks > 1 && !p.V.upper)) return "V.diag and V.upper are required";
    if (!p.P_r.diag) return "P_r.diag is required";
    if (p.XL.diag && !p.P_l.diag) return "P_l.diag is required for XL";
    if (p.XG.diag && !p.P_g.diag) return "P_g.diag is required for XG";
  }
  return "";
}

namespace {

struct BusyGuard {
  qtx_rgf_ctx* c;
  explicit BusyGuard(qtx_rgf_ctx* c_) : c(c_) { c->busy = true; }
  ~BusyGuard() { c->busy = false; }
};

}  // namespace

void qtx::run_lanes_to_end(qtx_rgf_ctx* c, std::vector<Lane*>& lanes) {
  const bool prof = (c->flags & QTX_FLAG_PROFILE) != 0;
  Executor& x = c->pool->exe(0);
  while (true) {
    x.build(lanes, kArenaLimit);
    if (x.empty()) break;
    x.flush(prof, c->graphs, c->stats);
  }
}

namespace {

qtx_status solve(qtx_rgf_ctx* c, qtx_rgf_problem* probs, int np) {
  const bool prof = (c->flags & QTX_FLAG_PROFILE) != 0;
  std::vector<Plan> plans(np);
  size_t n_e_tot = 0;
  std::vector<size_t> e_off(np);
  for (int i = 0; i < np; ++i) {
    probs[i].status = QTX_OK;
    probs[i].fail_energy = -1;
    probs[i].fail_block = -1;
    plans[i] = make_plan(probs[i]);
    e_off[i] = n_e_tot;
    n_e_tot += probs[i].n_energies;
  }
  // aux: energies | info
  const size_t eb = ((n_e_tot * 8) + 255) & ~size_t(255);
  const size_t ib = ((n_e_tot * 4) + 255) & ~size_t(255);
  ensure(c, &c->aux, &c->aux_bytes, eb + ib + 256);
  double* d_E = (double*)c->aux;
  int* d_info = (int*)(c->aux + eb);
  {
    std::vector<double> hE(n_e_tot, 0.0);
    for (int i = 0; i < np; ++i)
      if (probs[i].kind == QTX_KIND_G)
        std::memcpy(&hE[e_off[i]], probs[i].energies, sizeof(double) * probs[i].n_energies);
    HIPCHK(c, hipMemcpyAsync(d_E, hE.data(), sizeof(double) * n_e_tot, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }

  // lanes: the largest energy chunk whose workspace fits the budget
  const size_t budget = budget_now(c);
  struct Pend { int prob, e0, ec; size_t bytes; int part; };
  std::vector<Pend> pending;
  size_t total = 0, largest = 0;
  for (int i = 0; i < np; ++i) {
    const Plan& q = plans[i];
    if (lane_bytes(q, 1) > budget) {
      c->err = "problem " + std::to_string(i) + ": one energy needs " +
               std::to_string(lane_bytes(q, 1)) + " workspace bytes, budget is " + std::to_string(budget);
      throw Fail{QTX_ERR_NOMEM};
    }
    int lo = 1, hi = q.ne;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (lane_bytes(q, mid) <= budget) lo = mid; else hi = mid - 1;
    }
    // optionally a problem with many energies runs as `split` lanes on
    // different streams (one class each): while one lane is in its
    // latency-bound inverse, the other's products use the chip
    const int split = q.ne >= kSplitMinEnergies ? c->split : 1;
    if (split > 1) lo = std::min(lo, (q.ne + split - 1) / split);
    int chunk = 0;
    for (int e0 = 0; e0 < q.ne; e0 += lo, ++chunk) {
      const int ec = std::min(lo, q.ne - e0);
      const size_t by = lane_bytes(q, ec);
      pending.push_back(Pend{i, e0, ec, by, split > 1 ? chunk % split : 0});
      total += (by + 255) & ~size_t(255);
      largest = std::max(largest, by);
    }
  }
  const size_t cap = std::min(budget, total + 4096);
  ensure(c, &c->ws, &c->ws_bytes, std::max(cap, largest + 4096));

  // admission and merged execution: lanes are admitted in order while
  // their workspace fits; each goes to the executor (stream) of its shape
  // class, where lanes of the class share launches
  Regions reg(std::max(cap, largest + 4096));
  Pool& P = *c->pool;
  P.fork();
  std::map<uint64_t, int> spread;     // lanes admitted so far per spread class
  std::vector<std::unique_ptr<Lane>> active;
  std::vector<std::pair<Lane*, int>> fin;
  size_t next = 0;
  while (next < pending.size() || P.busy()) {
    while (next < pending.size()) {
      const Pend& pd = pending[next];
      size_t off = 0;
      if (!reg.alloc(pd.bytes, &off)) break;
      std::unique_ptr<Lane> L(new Lane());
      L->problem = pd.prob;
      L->e0 = pd.e0;
      L->ec = pd.ec;
      L->ws_off = off;
      L->ws_bytes = pd.bytes;
      const qtx_rgf_problem& p = probs[pd.prob];
      // lanes of one class (operation structure and block size) start
      // together and share one stream in lockstep; classes spread over the
      // pool's streams and overlap one another's latency-bound inverses
      const uint64_t base = lane_class(plans[pd.prob], p, c->batch_size_key);
      int part = pd.part;
      if (pd.ec <= kSpreadMaxEnergies && P.size() > 1 && pd.part == 0)
        part = spread[base]++ % std::min(P.size(), 8);
      const uint64_t cls = base * 8 + part;
      const int xi = P.place(cls);
      build_lane(*L, p, plans[pd.prob], c->ws + off, pd.e0, pd.ec, d_E + e_off[pd.prob],
                 d_info + e_off[pd.prob], c->tuner, P.stream(xi));
      L->cls = cls;                    // before add: the pool keys on it
      P.add(L.get(), xi);
      active.push_back(std::move(L));
      ++next;
    }
    if (!P.busy()) {
      c->err = "workspace admission stalled";
      throw Fail{QTX_ERR_NOMEM};
    }
    // with lanes waiting for memory, a segment stops once a lane finishes
    // so that its region is handed on promptly
    P.step(kArenaLimit, 1 << 30, next < pending.size(), prof, c->graphs, c->stats, fin);
    for (auto& f : fin) {
      reg.release(f.first->ws_off, f.first->ws_bytes);
      for (size_t i = 0; i < active.size(); ++i)
        if (active[i].get() == f.first) {
          active.erase(active.begin() + i);
          break;
        }
    }
    fin.clear();
  }
  P.join();
  std::vector<int> h_info(n_e_tot);
  HIPCHK(c, hipMemcpyAsync(h_info.data(), d_info, sizeof(int) * n_e_tot, hipMemcpyDeviceToHost, c->stream));
  P.sync_and_collect(c->stats);
  qtx_status worst = QTX_OK;
  for (int i = 0; i < np; ++i) {
    for (int e = 0; e < probs[i].n_energies; ++e) {
      const int v = h_info[e_off[i] + e];
      if (v != 0) {
        probs[i].status = v > 0 ? QTX_ERR_SINGULAR : QTX_ERR_NOT_FINITE;
        probs[i].fail_energy = e;
        probs[i].fail_block = std::abs(v) - 1;
        worst = QTX_ERR_PROBLEM;
        break;
      }
    }
  }
  return worst;
}

}  // namespace

extern "C" {

const char* qtx_rgf_status_string(qtx_status s) {
  switch (s) {
    case QTX_OK: return "ok";
    case QTX_ERR_INVALID_ARG: return "invalid argument";
    case QTX_ERR_SINGULAR: return "singular diagonal block (zero pivot)";
    case QTX_ERR_NOT_FINITE: return "non-finite pivot";
    case QTX_ERR_NOMEM: return "out of device memory / workspace budget";
    case QTX_ERR_HIP: return "HIP runtime error";
    case QTX_ERR_BUSY: return "context busy";
    case QTX_ERR_PROBLEM: return "at least one problem failed (see its status)";
  }
  return "unknown status";
}

const char* qtx_rgf_last_error(const qtx_rgf_ctx* c) { return c ? c->err.c_str() : ""; }

qtx_status qtx_rgf_create(qtx_rgf_ctx** out, int device, uint64_t budget, void* stream,
                          uint32_t flags) {
  if (!out) return QTX_ERR_INVALID_ARG;
  *out = nullptr;
  if (flags & ~QTX_FLAG_PROFILE) return QTX_ERR_INVALID_ARG;
  if (device < 0) return QTX_ERR_INVALID_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev) {
    (void)hipGetLastError();
    return QTX_ERR_HIP;
  }
  qtx_rgf_ctx* c = new (std::nothrow) qtx_rgf_ctx();
  if (!c) return QTX_ERR_NOMEM;
  c->device = device;
  c->budget = budget;
  c->flags = flags;
  const char* g = std::getenv("QTX_GRAPHS");
  c->graphs = !(g && g[0] == '0');
  const char* t = std::getenv("QTX_TUNE");
  c->tuner.set_enabled(!(t && t[0] == '0'));
  if (hipSetDevice(device) != hipSuccess) { delete c; return QTX_ERR_HIP; }
  // the allocation-free inverse's static scratch: its address on this device
  if (qtx::noalloc_init(device) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return QTX_ERR_HIP;
  }
  if (stream) {
    c->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return QTX_ERR_HIP;
    }
    c->own_stream = true;
  }
  const char* sp = std::getenv("QTX_SPLIT");
  if (sp) c->split = std::max(1, std::min(8, std::atoi(sp)));
  const char* bk = std::getenv("QTX_BATCH_CLASS");
  if (bk) c->batch_size_key = std::atoi(bk);
  const char* ns = std::getenv("QTX_STREAMS");
  int n_streams = ns ? std::atoi(ns) : 4;
  n_streams = std::max(1, std::min(8, n_streams));
  try {
    c->pool.reset(new Pool(c->stream, n_streams));
  } catch (const Fail&) {
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return QTX_ERR_HIP;
  }
  *out = c;
  return QTX_OK;
}

qtx_status qtx_rgf_destroy(qtx_rgf_ctx* c) {
  if (!c) return QTX_ERR_INVALID_ARG;
  if (c->busy) return QTX_ERR_BUSY;
  (void)hipSetDevice(c->device);
  qtx::stop_server(c);                   // drains the request loop first
  (void)hipStreamSynchronize(c->stream);
  c->pool.reset();
  if (c->ws) (void)hipFree(c->ws);
  if (c->aux) (void)hipFree(c->aux);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return QTX_OK;
}

qtx_status qtx_rgf_solve_batch(qtx_rgf_ctx* c, qtx_rgf_problem* probs, int32_t np) {
  if (!c) return QTX_ERR_INVALID_ARG;
  if (c->busy) return QTX_ERR_BUSY;
  c->err.clear();
  if (np < 0 || (np > 0 && !probs)) { c->err = "bad problem array"; return QTX_ERR_INVALID_ARG; }
  for (int i = 0; i < np; ++i) {
    const std::string m = validate_problem(probs[i]);
    if (!m.empty()) { c->err = "problem " + std::to_string(i) + ": " + m; return QTX_ERR_INVALID_ARG; }
  }
  if (np == 0) return QTX_OK;
  BusyGuard g(c);
  try {
    HIPCHK(c, hipSetDevice(c->device));
    return solve(c, probs, np);
  } catch (const Fail& f) {
    if (c->err.empty()) c->err = f.what;
    try { c->pool->sync_and_collect(c->stats); } catch (...) {}
    return (qtx_status)f.st;
  } catch (...) {
    c->err = "internal error";
    return QTX_ERR_HIP;
  }
}

double qtx_rgf_flops_per_energy(int32_t kind, int32_t n, int32_t b, int32_t n_rhs,
                                int32_t bt_rhs, int32_t want_wr) {
  if (n < 1 || b < 1 || n_rhs < 0) return 0.0;
  const double g = 8.0 * (double)b * b * b;
  const int per_fwd = 4 + (bt_rhs ? 1 : 0);
  const int per_bwd = 4 + (bt_rhs ? 3 : 0);
  double cnt = 1 + 2.0 * n_rhs + (n - 1.0) * (3 + per_fwd * n_rhs) + (n - 1.0) * (6 + per_bwd * n_rhs);
  if (kind == QTX_KIND_W) {
    // products of trunc(V P^R) and of the diagonal and upper blocks of
    // trunc(V P^s V^dag), both with block-tridiagonal P
    auto nprod = [&](int i, int j) {
      int c = 0;
      for (int k = std::max(0, i - 1); k <= std::min(n - 1, i + 1); ++k)
        if (std::abs(k - j) <= 1) ++c;
      return c;
    };
    double lhs = 0, rhs = 0;
    for (int i = 0; i < n; ++i) {
      for (int j = i - 1; j <= i + 1; ++j)
        if (j >= 0 && j < n) lhs += nprod(i, j);
      for (int k = i - 1; k <= i + 2; ++k)
        if (k >= 0 && k < n) rhs += nprod(i, k);
      for (int j = i; j <= i + 1; ++j) {
        if (j >= n) continue;
        for (int k = i - 1; k <= i + 2; ++k)
          if (k >= 0 && k < n && std::abs(k - j) <= 1) rhs += 1;
      }
    }
    cnt += lhs + n_rhs * rhs;
    if (want_wr) cnt += 3.0 * n - 2.0;          // (X^R V)_ii: 3 products, 1 at the ends
  }
  return cnt * g;
}

qtx_status qtx_rgf_kernel_stats(qtx_rgf_ctx* c, int32_t cls, int64_t* launches, double* ms,
                                double* flops, double* bytes) {
  if (!c || cls < 0 || cls >= kNumClasses) return QTX_ERR_INVALID_ARG;
  const KStat& s = c->stats[cls];
  if (launches) *launches = s.launches;
  if (ms) *ms = s.ms;
  if (flops) *flops = s.flops;
  if (bytes) *bytes = s.bytes;
  return QTX_OK;
}

qtx_status qtx_rgf_reset_stats(qtx_rgf_ctx* c) {
  if (!c) return QTX_ERR_INVALID_ARG;
  for (auto& s : c->stats) s = KStat();
  return QTX_OK;
}

}  // extern "C"

namespace {
qtx_status gemm_abi(bool fp32, qtx_rgf_ctx* c, char opa, char opb, int32_t m, int32_t n,
                    int32_t k, double ar, double ai, const void* A, int64_t lda, int64_t sA,
                    const void* B, int64_t ldb, int64_t sB, double br, double bi,
                    const void* C, int64_t ldc, int64_t sC, void* D, int64_t ldd, int64_t sD,
                    int32_t batch) {
  if (!c) return QTX_ERR_INVALID_ARG;
  if (c->busy) return QTX_ERR_BUSY;
  if ((opa != 'N' && opa != 'C') || (opb != 'N' && opb != 'C') || m < 0 || n < 0 || k < 0 ||
      batch < 0 || !A || !B || !D || (!C && (br != 0.0 || bi != 0.0)))
    return QTX_ERR_INVALID_ARG;
  const int64_t colsA = opa == 'N' ? k : m;
  const int64_t colsB = opb == 'N' ? n : k;
  if (lda < std::max<int64_t>(1, colsA) || ldb < std::max<int64_t>(1, colsB) ||
      ldd < std::max<int64_t>(1, n) || (C && ldc < std::max<int64_t>(1, n)))
    return QTX_ERR_INVALID_ARG;
  if (m == 0 || n == 0 || batch == 0) return QTX_OK;
  BusyGuard g(c);
  c->err.clear();
  try {
    HIPCHK(c, hipSetDevice(c->device));
    Lane L;
    GemmDesc d{};
    d.A = A; d.sA = sA; d.lda = lda;
    d.B = B; d.sB = sB; d.ldb = ldb;
    d.C = C; d.sC = sC; d.ldc = C ? ldc : ldd;
    d.D = D; d.sD = sD; d.ldd = ldd;
    d.alpha = zc{ar, ai};
    d.beta = C ? zc{br, bi} : zc{0.0, 0.0};
    d.M = m; d.N = n; d.K = k;
    d.batch = batch; d.batch2 = 1;
    L.gd.push_back(d);
    Op o;
    o.k = OpK::Gemm;
    o.opa = opa; o.opb = opb; o.fp32 = fp32;
    o.cfg = c->tuner.cfg(m, n, k, fp32, c->stream);
    o.first = 0; o.count = 1;
    o.flops = 8.0 * m * n * (double)k * batch;
    o.bytes = 16.0 * ((double)m * k + (double)k * n + (C ? 2.0 : 1.0) * m * n) * batch;
    L.ops.push_back(o);
    std::vector<Lane*> lp{&L};
    run_lanes_to_end(c, lp);
    c->pool->exe(0).sync_and_collect(c->stats);
  } catch (const Fail& f) {
    if (c->err.empty()) c->err = f.what;
    return (qtx_status)f.st;
  }
  return QTX_OK;
}
}  // namespace

extern "C" {

qtx_status qtx_rgf_zgemm(qtx_rgf_ctx* c, char opa, char opb, int32_t m, int32_t n, int32_t k,
                         double ar, double ai, const void* A, int64_t lda, int64_t sA,
                         const void* B, int64_t ldb, int64_t sB, double br, double bi,
                         const void* C, int64_t ldc, int64_t sC, void* D, int64_t ldd,
                         int64_t sD, int32_t batch) {
  return gemm_abi(false, c, opa, opb, m, n, k, ar, ai, A, lda, sA, B, ldb, sB, br, bi, C,
                  ldc, sC, D, ldd, sD, batch);
}

qtx_status qtx_rgf_cgemm(qtx_rgf_ctx* c, char opa, char opb, int32_t m, int32_t n, int32_t k,
                         double ar, double ai, const void* A, int64_t lda, int64_t sA,
                         const void* B, int64_t ldb, int64_t sB, double br, double bi,
                         const void* C, int64_t ldc, int64_t sC, void* D, int64_t ldd,
                         int64_t sD, int32_t batch) {
  return gemm_abi(true, c, opa, opb, m, n, k, ar, ai, A, lda, sA, B, ldb, sB, br, bi, C,
                  ldc, sC, D, ldd, sD, batch);
}

qtx_status qtx_rgf_zinv(qtx_rgf_ctx* c, int32_t b, void* A, void* X, int32_t* info,
                        int32_t batch) {
  if (!c || b < 1 || b > kMaxB || !A || !X || batch < 0 || A == X) return QTX_ERR_INVALID_ARG;
  if (c->busy) return QTX_ERR_BUSY;
  if (batch == 0) return QTX_OK;
  BusyGuard g(c);
  c->err.clear();
  void* work = nullptr;
  try {
    HIPCHK(c, hipSetDevice(c->device));
    // (the one-launch inverse for b <= kSmallB uses no work buffers)
    const bool small = b <= kSmallB;
    const size_t pan = small ? 0 : (size_t)batch * b * kPanel * 16;
    const size_t span = small ? 0 : (size_t)batch * b * inv_span(b) * 16;
    const size_t ints = small ? 0 : (size_t)batch * b * 4;
    HIPCHK(c, hipMalloc(&work, 2 * pan + 2 * span + 2 * ints + 4096));
    Lane L;
    InvDesc d{};
    d.S = A; d.sS = (long long)b * b;
    d.X = X; d.sX = (long long)b * b;
    char* w = (char*)work;
    d.panel = w;
    d.brow = w + pan;
    d.spanel = w + 2 * pan;
    d.sbrow = w + 2 * pan + span;
    d.perm = (int*)(w + 2 * pan + 2 * span);
    d.used = (int*)(w + 2 * pan + 2 * span + ints);
    d.info = info; d.code = 0; d.reset_info = 1;
    d.b = b; d.batch = batch;
    L.id.push_back(d);
    Op o;
    o.k = OpK::Inv;
    o.first = 0; o.count = 1;
    o.flops = 8.0 * (double)b * b * b * batch;
    L.ops.push_back(o);
    std::vector<Lane*> lp{&L};
    run_lanes_to_end(c, lp);
    c->pool->exe(0).sync_and_collect(c->stats);
    HIPCHK(c, hipFree(work));
  } catch (const Fail& f) {
    if (c->err.empty()) c->err = f.what;
    if (work) (void)hipFree(work);
    return (qtx_status)f.st;
  }
  return QTX_OK;
}

}  // extern "C"

namespace {

// One lane of batched b x b complex128 operations for the lead solvers; all
// energies advance together in merged launches, in the order pushed.
struct LeadLane {
  Lane L;
  int b, batch, cfg;
  long long bb;
  char* iw;                    // inverse work buffers for `batch` matrices
  size_t pan, span, ints;

  LeadLane(qtx_rgf_ctx* c, int b_, int batch_, char* inv_work)
      : b(b_), batch(batch_), bb((long long)b_ * b_), iw(inv_work) {
    cfg = c->tuner.cfg(b, b, b, false, c->stream);
    pan = (size_t)batch * b * kPanel * 16;
    span = (size_t)batch * b * inv_span(b) * 16;
    ints = (size_t)batch * b * 4;
  }
  static size_t inv_work(int b, int batch) {
    return (size_t)batch * b * (2 * kPanel + 2 * inv_span(b)) * 16 + (size_t)batch * b * 8 + 4096;
  }
  // D = alpha op(A) op(B) + beta C (strides in elements between energies;
  // op 'C' = adjoint)
  void gemm(const void* A, long long sA, const void* B, long long sB, const void* C,
            long long sC, void* D, double alpha, double beta, char opa = 'N',
            char opb = 'N') {
    GemmDesc d{};
    d.A = A; d.sA = sA; d.lda = b;
    d.B = B; d.sB = sB; d.ldb = b;
    d.C = C; d.sC = sC; d.ldc = b;
    d.D = D; d.sD = bb; d.ldd = b;
    d.alpha = zc{alpha, 0.0};
    d.beta = C ? zc{beta, 0.0} : zc{0.0, 0.0};
    d.M = b; d.N = b; d.K = b;
    d.batch = batch; d.batch2 = 1;
    L.gd.push_back(d);
    Op o;
    o.k = OpK::Gemm;
    o.opa = opa; o.opb = opb; o.fp32 = false;
    o.cfg = cfg;
    o.first = (int)L.gd.size() - 1; o.count = 1;
    o.flops = 8.0 * (double)bb * b * batch;
    o.bytes = 16.0 * (C ? 4.0 : 3.0) * (double)bb * batch;
    L.ops.push_back(o);
  }
  // X = S^{-1} (S is overwritten); info keeps the first failure's code
  void inv(void* S, void* X, int* info, int code, bool reset_info) {
    InvDesc d{};
    d.S = S; d.sS = bb;
    d.X = X; d.sX = bb;
    d.panel = iw;
    d.brow = iw + pan;
    d.spanel = iw + 2 * pan;
    d.sbrow = iw + 2 * pan + span;
    d.perm = (int*)(iw + 2 * pan + 2 * span);
    d.used = (int*)(iw + 2 * pan + 2 * span + ints);
    d.info = info; d.code = code; d.reset_info = reset_info ? 1 : 0;
    d.b = b; d.batch = batch;
    L.id.push_back(d);
    Op o;
    o.k = OpK::Inv;
    o.first = (int)L.id.size() - 1; o.count = 1;
    o.flops = 8.0 * (double)bb * b * batch;
    L.ops.push_back(o);
  }
  // D = c0 S0 + c1 S1 (S1 may be null)
  void lin(const void* s0, long long ss0, double c0, const void* s1, long long ss1, double c1,
           void* D) {
    LinCombDesc a{};
    a.src[0] = s0; a.sSrc[0] = ss0; a.c[0] = zc{c0, 0.0};
    a.src[1] = s1; a.sSrc[1] = ss1; a.c[1] = zc{c1, 0.0};
    a.D = D; a.sD = bb;
    a.b = b; a.batch = batch;
    L.ld.push_back(a);
    Op o;
    o.k = OpK::Lin;
    o.first = (int)L.ld.size() - 1; o.count = 1;
    o.bytes = 16.0 * (double)bb * batch * (2 + (s1 != nullptr));
    L.ops.push_back(o);
  }
};

// Byte range [lo, hi) of `batch` b x b complex128 blocks at stride s
// elements (0 = one shared block).
struct Span {
  uintptr_t lo, hi;
};
Span span_of(const void* p, long long bb, int64_t s, int batch) {
  const uintptr_t lo = (uintptr_t)p;
  const long long last = (s == 0 || batch <= 1) ? 0 : (long long)(batch - 1) * s;
  return Span{lo, lo + (uintptr_t)((last + bb) * 16)};
}
bool overlap(const Span& a, const Span& b) { return a.lo < b.hi && b.lo < a.hi; }

qtx_status lead_args_ok(int32_t b, int32_t batch, const void* m, int64_t s_m, const void* n,
                        int64_t s_n, const void* n_prime, int64_t s_np, const void* x,
                        int32_t count) {
  if (b < 1 || b > 1024 || batch < 0 || count < 1 || !m || !n || !n_prime || !x)
    return QTX_ERR_INVALID_ARG;
  const long long bb = (long long)b * b;
  auto bad_stride = [bb](int64_t st) { return st != 0 && st < bb; };
  if (bad_stride(s_m) || bad_stride(s_n) || bad_stride(s_np)) return QTX_ERR_INVALID_ARG;
  return QTX_OK;
}

}  // namespace

extern "C" {

// Eq. (naive) for all energies at once: one lane holding the n_iter
// iterations (two products and one inverse each) and the boundary block, so
// the whole chain runs as merged launches with no host round trip.
qtx_status qtx_rgf_obc_fixed_point(qtx_rgf_ctx* c, int32_t b, int32_t batch, const void* m,
                                   int64_t s_m, const void* n, int64_t s_n, const void* n_prime,
                                   int64_t s_np, void* x, void* sigma, double* update,
                                   int32_t* info, int32_t n_iter) {
  if (!c) return QTX_ERR_INVALID_ARG;
  if (!info) return QTX_ERR_INVALID_ARG;
  const qtx_status ok = lead_args_ok(b, batch, m, s_m, n, s_n, n_prime, s_np, x, n_iter);
  if (ok != QTX_OK) return ok;
  {
    const long long bb = (long long)b * b;
    const Span in[3] = {span_of(m, bb, s_m, batch), span_of(n, bb, s_n, batch),
                        span_of(n_prime, bb, s_np, batch)};
    const Span sx = span_of(x, bb, bb, batch);
    for (const Span& r : in)
      if (overlap(sx, r) || (sigma && overlap(span_of(sigma, bb, bb, batch), r)))
        return QTX_ERR_INVALID_ARG;
    if (sigma && overlap(sx, span_of(sigma, bb, bb, batch))) return QTX_ERR_INVALID_ARG;
  }
  if (c->busy) return QTX_ERR_BUSY;
  if (batch == 0) return QTX_OK;
  BusyGuard g(c);
  c->err.clear();
  char* work = nullptr;
  try {
    HIPCHK(c, hipSetDevice(c->device));
    const long long bb = (long long)b * b;
    const size_t blk = (size_t)batch * bb * 16;
    const size_t iwb = LeadLane::inv_work(b, batch);
    ensure(c, &c->ws, &c->ws_bytes, 3 * blk + iwb + norm_scratch_bytes(bb, batch));   // grow-only
    work = c->ws;
    double* part = (double*)(work + 3 * blk + iwb);
    void* T = work;
    void* W = work + blk;
    void* xb = work + 2 * blk;
    LeadLane q(c, b, batch, work + 3 * blk);
    void* cur = x;
    void* nxt = xb;
    for (int it = 0; it < n_iter; ++it) {
      q.gemm(cur, bb, n_prime, s_np, nullptr, 0, T, 1.0, 0.0);       // T = x_i n'
      q.gemm(n, s_n, T, bb, m, s_m, W, -1.0, 1.0);                   // W = m - n T
      q.inv(W, nxt, info, it + 1, it == 0);                          // x_{i+1} = W^{-1}
      std::swap(cur, nxt);
    }
    // cur = x_N, nxt = x_{N-1}
    if (sigma) {
      q.gemm(cur, bb, n_prime, s_np, nullptr, 0, T, 1.0, 0.0);
      q.gemm(n, s_n, T, bb, nullptr, 0, sigma, 1.0, 0.0);
    }
    std::vector<Lane*> lp{&q.L};
    run_lanes_to_end(c, lp);
    const hipStream_t st = c->pool->exe(0).stream();
    if (update) HIPCHK(c, launch_update_norm(cur, nxt, update, bb, batch, part, st));
    if (cur != x) HIPCHK(c, hipMemcpyAsync(x, cur, blk, hipMemcpyDeviceToDevice, st));
    c->pool->exe(0).sync_and_collect(c->stats);
  } catch (const Fail& f) {
    if (c->err.empty()) c->err = f.what;
    return (qtx_status)f.st;
  }
  return QTX_OK;
}

// Sancho-Rubio decimation for all energies at once: each step copies the
// bulk block (the inverse overwrites its input), inverts it, forms
// n g n' once and folds it into both the surface and the bulk blocks, and
// squares the couplings; then x = m_surf^{-1} and n x n'.
qtx_status qtx_rgf_obc_sancho_rubio(qtx_rgf_ctx* c, int32_t b, int32_t batch, const void* m,
                                    int64_t s_m, const void* n, int64_t s_n,
                                    const void* n_prime, int64_t s_np, void* x, void* sigma,
                                    double* coupling, int32_t* info, int32_t n_steps) {
  if (!c) return QTX_ERR_INVALID_ARG;
  if (!info) return QTX_ERR_INVALID_ARG;
  const qtx_status ok = lead_args_ok(b, batch, m, s_m, n, s_n, n_prime, s_np, x, n_steps);
  if (ok != QTX_OK) return ok;
  {
    const long long bb = (long long)b * b;
    const Span in[3] = {span_of(m, bb, s_m, batch), span_of(n, bb, s_n, batch),
                        span_of(n_prime, bb, s_np, batch)};
    const Span sx = span_of(x, bb, bb, batch);
    for (const Span& r : in)
      if (overlap(sx, r) || (sigma && overlap(span_of(sigma, bb, bb, batch), r)))
        return QTX_ERR_INVALID_ARG;
    if (sigma && overlap(sx, span_of(sigma, bb, bb, batch))) return QTX_ERR_INVALID_ARG;
  }
  if (c->busy) return QTX_ERR_BUSY;
  if (batch == 0) return QTX_OK;
  BusyGuard g(c);
  c->err.clear();
  char* work = nullptr;
  try {
    HIPCHK(c, hipSetDevice(c->device));
    const long long bb = (long long)b * b;
    const size_t blk = (size_t)batch * bb * 16;
    constexpr int kBlocks = 11;
    const size_t iwb = LeadLane::inv_work(b, batch);
    ensure(c, &c->ws, &c->ws_bytes, kBlocks * blk + iwb + norm_scratch_bytes(bb, batch));
    work = c->ws;                                   // grow-only, reused
    double* part = (double*)(work + kBlocks * blk + iwb);
    char* w = work;
    void* ms = w;            void* mb = w + blk;       void* W = w + 2 * blk;
    void* gi = w + 3 * blk;  void* ga = w + 4 * blk;   void* gc = w + 5 * blk;
    void* T = w + 6 * blk;
    void* a2[2] = {w + 7 * blk, w + 8 * blk};
    void* c2[2] = {w + 9 * blk, w + 10 * blk};
    LeadLane q(c, b, batch, work + kBlocks * blk);
    const void* a = n;         long long sa = s_n;
    const void* cp = n_prime;  long long sc = s_np;
    const void* msrc = m;      long long sms = s_m;    // surface block so far
    const void* mbsrc = m;     long long smb = s_m;    // bulk block so far
    for (int k = 0; k < n_steps; ++k) {
      q.lin(mbsrc, smb, 1.0, nullptr, 0, 0.0, W);                  // W = m_bulk
      q.inv(W, gi, info, k + 1, k == 0);                           // g = m_bulk^{-1}
      q.gemm(gi, bb, a, sa, nullptr, 0, ga, 1.0, 0.0);             // g n
      q.gemm(gi, bb, cp, sc, nullptr, 0, gc, 1.0, 0.0);            // g n'
      q.gemm(a, sa, gc, bb, nullptr, 0, T, 1.0, 0.0);              // T = n g n'
      q.lin(msrc, sms, 1.0, T, bb, -1.0, ms);                      // m_surf -= T
      q.lin(mbsrc, smb, 1.0, T, bb, -1.0, mb);                     // m_bulk -= T
      q.gemm(cp, sc, ga, bb, mb, bb, mb, -1.0, 1.0);               // m_bulk -= n' g n
      void* an = a2[k & 1];
      void* cn = c2[k & 1];
      q.gemm(a, sa, ga, bb, nullptr, 0, an, -1.0, 0.0);            // n <- -n g n
      q.gemm(cp, sc, gc, bb, nullptr, 0, cn, -1.0, 0.0);           // n' <- -n' g n'
      a = an; sa = bb;
      cp = cn; sc = bb;
      msrc = ms; sms = bb;
      mbsrc = mb; smb = bb;
    }
    q.lin(ms, bb, 1.0, nullptr, 0, 0.0, W);
    q.inv(W, x, info, n_steps + 1, false);                         // x = m_surf^{-1}
    if (sigma) {
      q.gemm(x, bb, n_prime, s_np, nullptr, 0, T, 1.0, 0.0);
      q.gemm(n, s_n, T, bb, nullptr, 0, sigma, 1.0, 0.0);
    }
    std::vector<Lane*> lp{&q.L};
    run_lanes_to_end(c, lp);
    const hipStream_t st = c->pool->exe(0).stream();
    if (coupling)
      HIPCHK(c, launch_coupling_norm(a, cp, n, s_n, n_prime, s_np, coupling, bb, batch, part,
                                     st));
    c->pool->exe(0).sync_and_collect(c->stats);
  } catch (const Fail& f) {
    if (c->err.empty()) c->err = f.what;
    return (qtx_status)f.st;
  }
  return QTX_OK;
}

// Both outputs in one pass over the retarded blocks: the per-energy
// occupations go to the device once, then one launch over (energy, tile).
qtx_status qtx_rgf_obc_lesser_greater(qtx_rgf_ctx* c, int32_t b, int32_t batch,
                                      const void* sigma_r, int64_t s_sr, const double* f,
                                      const double* one_minus_f, void* sigma_l,
                                      void* sigma_g) {
  if (!c || b < 1 || b > 1024 || batch < 0 || !sigma_r || (!sigma_l && !sigma_g))
    return QTX_ERR_INVALID_ARG;
  if ((sigma_l && !f) || (sigma_g && !one_minus_f)) return QTX_ERR_INVALID_ARG;
  const long long bb = (long long)b * b;
  if (s_sr != 0 && s_sr < bb) return QTX_ERR_INVALID_ARG;
  if (batch > 0) {
    const Span in = span_of(sigma_r, bb, s_sr, batch);
    if ((sigma_l && overlap(span_of(sigma_l, bb, bb, batch), in)) ||
        (sigma_g && overlap(span_of(sigma_g, bb, bb, batch), in)) ||
        (sigma_l && sigma_g &&
         overlap(span_of(sigma_l, bb, bb, batch), span_of(sigma_g, bb, bb, batch))))
      return QTX_ERR_INVALID_ARG;
  }
  if (c->busy) return QTX_ERR_BUSY;
  if (batch == 0) return QTX_OK;
  BusyGuard g(c);
  c->err.clear();
  try {
    HIPCHK(c, hipSetDevice(c->device));
    std::vector<double> occ(2 * (size_t)batch);
    for (int e = 0; e < batch; ++e) {
      occ[2 * (size_t)e] = f ? f[e] : 0.0;
      occ[2 * (size_t)e + 1] = one_minus_f ? one_minus_f[e] : 0.0;
    }
    ensure(c, &c->aux, &c->aux_bytes, occ.size() * sizeof(double) + 256);
    const hipStream_t st = c->pool->exe(0).stream();
    HIPCHK(c, hipMemcpyAsync(c->aux, occ.data(), occ.size() * sizeof(double),
                             hipMemcpyHostToDevice, st));
    HIPCHK(c, launch_lesser_greater(sigma_r, s_sr, (const double*)c->aux, sigma_l, sigma_g, b,
                                    batch, st));
    c->pool->exe(0).sync_and_collect(c->stats);
  } catch (const Fail& fl) {
    if (c->err.empty()) c->err = fl.what;
    return (qtx_status)fl.st;
  }
  return QTX_OK;
}

// Observables: H_{i,i+1}^dagger for every interface once (adjoint kernel),
// then one reduction launch over (energy, block or interface).
qtx_status qtx_rgf_observables(qtx_rgf_ctx* c, int32_t n_blocks, int32_t b, int32_t batch,
                               const void* XL_diag, const void* XG_diag, const void* XL_lower,
                               const void* H_upper, double* dos, double* density,
                               double* current) {
  if (!c || b < 1 || b > 1024 || n_blocks < 1 || batch < 0 || !XL_diag) return QTX_ERR_INVALID_ARG;
  if (dos && !XG_diag) return QTX_ERR_INVALID_ARG;
  const bool want_cur = current && n_blocks > 1;
  if (want_cur && (!XL_lower || !H_upper)) return QTX_ERR_INVALID_ARG;
  if (!dos && !density && !current) return QTX_ERR_INVALID_ARG;
  if (c->busy) return QTX_ERR_BUSY;
  if (batch == 0) return QTX_OK;
  BusyGuard g(c);
  c->err.clear();
  void* hd = nullptr;
  try {
    HIPCHK(c, hipSetDevice(c->device));
    const long long bb = (long long)b * b;
    const hipStream_t st = c->pool->exe(0).stream();
    double* part = nullptr;
    if (want_cur) {
      // the couplings' adjoints, then the current's partial sums
      const size_t hd_bytes = ((size_t)(n_blocks - 1) * bb * 16 + 255) & ~(size_t)255;
      ensure(c, &c->ws, &c->ws_bytes, hd_bytes + observables_part_bytes(n_blocks, b, batch));
      hd = c->ws;
      part = (double*)(c->ws + hd_bytes);
      Lane L;
      TransDesc t{};
      t.C = nullptr;
      t.Z = H_upper;
      t.D = hd;
      t.sC = 0; t.sZ = bb; t.sD = bb;
      t.a = zc{0.0, 0.0};
      t.z = zc{0.0, 0.0};
      t.g = zc{1.0, 0.0};                      // D = Z^dagger
      t.b = b; t.batch = n_blocks - 1;
      L.td.push_back(t);
      Op o;
      o.k = OpK::Trans;
      o.first = 0; o.count = 1;
      o.bytes = 32.0 * (double)bb * (n_blocks - 1);
      L.ops.push_back(o);
      std::vector<Lane*> lp{&L};
      run_lanes_to_end(c, lp);
    }
    HIPCHK(c, launch_observables(XL_diag, XG_diag, want_cur ? XL_lower : nullptr, hd, dos,
                                 density, want_cur ? current : nullptr, n_blocks, b, batch,
                                 part, st));
    c->pool->exe(0).sync_and_collect(c->stats);
  } catch (const Fail& fl) {
    if (c->err.empty()) c->err = fl.what;
    return (qtx_status)fl.st;
  }
  return QTX_OK;
}

// Eq. (interaction): the element-wise energy convolution, one launch.
qtx_status qtx_rgf_energy_convolution(qtx_rgf_ctx* c, int64_t n_elem, const void* X1,
                                      int32_t n1, int32_t reverse1, const void* X2, int32_t n2,
                                      void* B, int32_t n_out, int32_t shift, double scale_re,
                                      double scale_im) {
  if (!c || n_elem < 0 || n1 < 1 || n2 < 1 || n_out < 0 || !X1 || !X2 || !B)
    return QTX_ERR_INVALID_ARG;
  if (reverse1 != 0 && reverse1 != 1) return QTX_ERR_INVALID_ARG;
  {
    const Span sb = span_of(B, n_elem, n_elem, n_out);
    if (overlap(sb, span_of(X1, n_elem, n_elem, n1)) || overlap(sb, span_of(X2, n_elem, n_elem, n2)))
      return QTX_ERR_INVALID_ARG;
  }
  if (c->busy) return QTX_ERR_BUSY;
  if (n_elem == 0 || n_out == 0) return QTX_OK;
  BusyGuard g(c);
  c->err.clear();
  try {
    HIPCHK(c, hipSetDevice(c->device));
    const hipStream_t st = c->pool->exe(0).stream();
    HIPCHK(c, launch_energy_convolution(X1, n1, reverse1, X2, n2, B, n_out, shift, scale_re,
                                        scale_im, n_elem, st));
    HIPCHK(c, hipStreamSynchronize(st));
  } catch (const Fail& fl) {
    if (c->err.empty()) c->err = fl.what;
    return (qtx_status)fl.st;
  }
  return QTX_OK;
}

// Eq. (lyapunov) by the plain iteration, all energies at once: two
// products per iteration (T = w a^dagger, w' = q - a T), ping-pong buffers.
qtx_status qtx_rgf_obc_lyapunov_fixed_point(qtx_rgf_ctx* c, int32_t b, int32_t batch,
                                            const void* a, int64_t s_a, const void* q,
                                            int64_t s_q, void* w, double* update,
                                            int32_t n_iter) {
  if (!c) return QTX_ERR_INVALID_ARG;
  const qtx_status ok = lead_args_ok(b, batch, a, s_a, q, s_q, q, s_q, w, n_iter);
  if (ok != QTX_OK) return ok;
  {
    const long long bb = (long long)b * b;
    const Span sw = span_of(w, bb, bb, batch);
    if (overlap(sw, span_of(a, bb, s_a, batch)) || overlap(sw, span_of(q, bb, s_q, batch)))
      return QTX_ERR_INVALID_ARG;
  }
  if (c->busy) return QTX_ERR_BUSY;
  if (batch == 0) return QTX_OK;
  BusyGuard g(c);
  c->err.clear();
  char* work = nullptr;
  try {
    HIPCHK(c, hipSetDevice(c->device));
    const long long bb = (long long)b * b;
    const size_t blk = (size_t)batch * bb * 16;
    ensure(c, &c->ws, &c->ws_bytes, 2 * blk + norm_scratch_bytes(bb, batch));   // grow-only
    work = c->ws;
    double* part = (double*)(work + 2 * blk);
    void* T = work;
    void* wb = work + blk;
    LeadLane lane(c, b, batch, nullptr);
    void* cur = w;
    void* nxt = wb;
    for (int it = 0; it < n_iter; ++it) {
      lane.gemm(cur, bb, a, s_a, nullptr, 0, T, 1.0, 0.0, 'N', 'C');   // T = w a^dagger
      lane.gemm(a, s_a, T, bb, q, s_q, nxt, -1.0, 1.0);               // w' = q - a T
      std::swap(cur, nxt);
    }
    std::vector<Lane*> lp{&lane.L};
    run_lanes_to_end(c, lp);
    const hipStream_t st = c->pool->exe(0).stream();
    if (update) HIPCHK(c, launch_update_norm(cur, nxt, update, bb, batch, part, st));
    if (cur != w) HIPCHK(c, hipMemcpyAsync(w, cur, blk, hipMemcpyDeviceToDevice, st));
    c->pool->exe(0).sync_and_collect(c->stats);
  } catch (const Fail& fl) {
    if (c->err.empty()) c->err = fl.what;
    return (qtx_status)fl.st;
  }
  return QTX_OK;
}

// Eq. (lyapunov) by doubling, all energies at once: S_1 = q - a q a^dagger,
// then per step A <- A A and S <- S + A S A^dagger (three products).
qtx_status qtx_rgf_obc_lyapunov_doubling(qtx_rgf_ctx* c, int32_t b, int32_t batch,
                                         const void* a, int64_t s_a, const void* q,
                                         int64_t s_q, void* w, double* remaining,
                                         int32_t n_steps) {
  if (!c) return QTX_ERR_INVALID_ARG;
  const qtx_status ok = lead_args_ok(b, batch, a, s_a, q, s_q, q, s_q, w, n_steps);
  if (ok != QTX_OK) return ok;
  {
    const long long bb = (long long)b * b;
    const Span sw = span_of(w, bb, bb, batch);
    if (overlap(sw, span_of(a, bb, s_a, batch)) || overlap(sw, span_of(q, bb, s_q, batch)))
      return QTX_ERR_INVALID_ARG;
  }
  if (c->busy) return QTX_ERR_BUSY;
  if (batch == 0) return QTX_OK;
  BusyGuard g(c);
  c->err.clear();
  char* work = nullptr;
  try {
    HIPCHK(c, hipSetDevice(c->device));
    const long long bb = (long long)b * b;
    const size_t blk = (size_t)batch * bb * 16;
    ensure(c, &c->ws, &c->ws_bytes, 3 * blk + norm_scratch_bytes(bb, batch));   // grow-only
    work = c->ws;
    double* part = (double*)(work + 3 * blk);
    void* T = work;
    void* A2[2] = {work + blk, work + 2 * blk};
    LeadLane lane(c, b, batch, nullptr);
    lane.gemm(q, s_q, a, s_a, nullptr, 0, T, 1.0, 0.0, 'N', 'C');      // T = q a^dagger
    lane.gemm(a, s_a, T, bb, q, s_q, w, -1.0, 1.0);                    // S = q - a T
    const void* A = a;
    long long sA = s_a;
    for (int k = 1; k <= n_steps; ++k) {
      void* An = A2[k & 1];
      lane.gemm(A, sA, A, sA, nullptr, 0, An, 1.0, 0.0);               // A <- A A
      A = An;
      sA = bb;
      if (k == n_steps) break;                 // the last square only measures
      lane.gemm(w, bb, A, sA, nullptr, 0, T, 1.0, 0.0, 'N', 'C');      // T = S A^dagger
      lane.gemm(A, sA, T, bb, w, bb, w, 1.0, 1.0);                     // S += A T
    }
    std::vector<Lane*> lp{&lane.L};
    run_lanes_to_end(c, lp);
    const hipStream_t st = c->pool->exe(0).stream();
    if (remaining)
      HIPCHK(c, launch_coupling_norm(A, A, a, s_a, a, s_a, remaining, bb, batch, part, st));
    c->pool->exe(0).sync_and_collect(c->stats);
  } catch (const Fail& fl) {
    if (c->err.empty()) c->err = fl.what;
    return (qtx_status)fl.st;
  }
  return QTX_OK;
}

}  // extern "C"
