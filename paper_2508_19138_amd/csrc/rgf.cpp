// C ABI and host orchestration of the batched RGF selected inversion
// (arXiv 2508.19138, Sec. 3.2.3, Eqs. forward-pass / backward-pass).
//
// One problem's energies are processed in chunks that fit the workspace
// budget.  Every step of the recursion is a handful of grouped, strided-
// batched launches over all energies of the chunk: complex products on the
// FP64 matrix cores (zgemm), the blocked Gauss-Jordan inverse (zinv), and
// elementwise assembly / anti-Hermitian updates.  Operand roles follow the
// paper: x_i = x^R_i (left-connected), xs_i = x^s_i, X_i = X^R_i, with
// U_i = Mt_{i,i+1}, L_i = Mt_{i+1,i}.  Right-hand sides are anti-Hermitian,
// so  y - y^dag,  Y - Y^dag  and  Z - Z^dag  each need one product, and the
// lower blocks of X^s are -upper^dagger.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/qtx_rgf.h"
#include "qtx_internal.h"

using namespace qtx;

namespace {

constexpr int kClassZgemm = 0, kClassCgemm = 1, kClassInv = 2, kClassElem = 3;
constexpr int kNumClasses = 4;

struct KStat {
  int64_t launches = 0;
  double ms = 0, flops = 0, bytes = 0;
};
struct Pending {
  int cls;
  hipEvent_t a, b;
  double flops, bytes;
};

}  // namespace

struct qtx_rgf_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  uint64_t budget = 0;
  uint32_t flags = 0;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  std::string err;
  KStat stats[kNumClasses];
  std::vector<hipEvent_t> ev_pool;
  std::vector<Pending> pending;
  bool busy = false;
};

namespace {

const zc kOne{1.0, 0.0}, kZero{0.0, 0.0}, kMinus{-1.0, 0.0};
inline zc rs(double v) { return zc{v, 0.0}; }

struct Fail {
  qtx_status st;
};

#define HIPCHK(ctx, expr)                                                    \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess) {                                                  \
      (ctx)->err = std::string(#expr) + ": " + hipGetErrorString(e_);        \
      throw Fail{QTX_ERR_HIP};                                               \
    }                                                                        \
  } while (0)

hipEvent_t get_event(qtx_rgf_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIPCHK(c, hipEventCreate(&e));
  return e;
}

void flush_stats(qtx_rgf_ctx* c) {
  for (auto& p : c->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      KStat& s = c->stats[p.cls];
      s.launches += 1;
      s.ms += ms;
      s.flops += p.flops;
      s.bytes += p.bytes;
    }
    c->ev_pool.push_back(p.a);
    c->ev_pool.push_back(p.b);
  }
  c->pending.clear();
}

template <class F>
void timed(qtx_rgf_ctx* c, int cls, double flops, double bytes, F&& f) {
  if (!(c->flags & QTX_FLAG_PROFILE)) {
    HIPCHK(c, f());
    return;
  }
  hipEvent_t a = get_event(c), b = get_event(c);
  HIPCHK(c, hipEventRecord(a, c->stream));
  HIPCHK(c, f());
  HIPCHK(c, hipEventRecord(b, c->stream));
  c->pending.push_back(Pending{cls, a, b, flops, bytes});
  if (c->pending.size() > 4096) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    flush_stats(c);
  }
}

// A block-indexed operand: block i of energy e (relative to the view's
// base) starts at p + e * es + i * bs (complex elements).
struct View {
  const double2* p = nullptr;
  long long es = 0, bs = 0;
  bool ok() const { return p != nullptr; }
  const double2* at(long long i) const { return p + i * bs; }
  double2* w(long long i) const { return const_cast<double2*>(p + i * bs); }
};

// One operand of a product: a block of a view, optionally adjoint.
struct Opnd {
  View v;
  long long i;
};

struct Term {            // D = alpha * A B + beta * C, all views batched over e
  Opnd A, B;
  const View* C;         // null = no C
  long long ic;
  View D;
  long long id;
  zc alpha, beta;
};

class Solver {
 public:
  Solver(qtx_rgf_ctx* c, int b, int ec) : c_(c), b_(b), ec_(ec) {
    blk_ = (long long)b * b;
  }
  // QTX_MIXED: the recursion's products run on the FP32 matrix cores with
  // FP64 epilogues; inverses, assembly and storage stay FP64.
  void set_fp32_products(bool on) { fp32_ = on; }

  // Grouped product launch: all terms share op and shape (b x b x b),
  // the batch is the chunk's energies, and `nb2` consecutive blocks
  // (stride = each view's bs) form the second batch index.
  void gemm(char opa, char opb, std::initializer_list<Term> terms, int nb2 = 1,
            int m = -1, int n = -1, int k = -1) {
    GemmArgs g{};
    g.M = m < 0 ? b_ : m;
    g.N = n < 0 ? b_ : n;
    g.K = k < 0 ? b_ : k;
    g.lda = b_; g.ldb = b_; g.ldc = b_; g.ldd = b_;
    g.batch = ec_;
    g.batch2 = nb2;
    g.ngroups = 0;
    double bytes = 0;
    for (const Term& t : terms) {
      GemmGroup& q = g.g[g.ngroups++];
      q.A = t.A.v.at(t.A.i); q.sA = t.A.v.es; q.tA = t.A.v.bs;
      q.B = t.B.v.at(t.B.i); q.sB = t.B.v.es; q.tB = t.B.v.bs;
      if (t.C) { q.C = t.C->at(t.ic); q.sC = t.C->es; q.tC = t.C->bs; }
      else { q.C = nullptr; q.sC = 0; q.tC = 0; }
      q.D = t.D.w(t.id); q.sD = t.D.es; q.tD = t.D.bs;
      q.alpha = t.alpha;
      q.beta = t.C ? t.beta : kZero;
      bytes += 16.0 * ((double)g.M * g.K + (double)g.K * g.N +
                       (t.C ? 2.0 : 1.0) * g.M * g.N);
    }
    const double mult = (double)ec_ * nb2;
    const double flops = 8.0 * g.M * g.N * (double)g.K * g.ngroups * mult;
    if (fp32_)
      timed(c_, kClassCgemm, flops, bytes * mult, [&] { return launch_cgemm(opa, opb, g, c_->stream); });
    else
      timed(c_, kClassZgemm, flops, bytes * mult, [&] { return launch_zgemm(opa, opb, g, c_->stream); });
  }

  void inverse(const View& S, long long is, const View& X, long long ix,
               const InvWork& w, int* info, int code) {
    const double fl = 8.0 * (double)b_ * b_ * b_ * ec_;
    const double by = 16.0 * 2.0 * blk_ * ec_ * ((b_ + kPanel - 1) / kPanel);
    timed(c_, kClassInv, fl, by, [&] {
      return launch_zinv(b_, S.w(is), S.es, X.w(ix), X.es, ec_, w, info, code, c_->stream);
    });
  }

  void lincomb(const LinComb& a) {
    const double by = 16.0 * blk_ * ec_ * (1 + (a.src[0] != nullptr) + (a.src[1] != nullptr) + (a.src[2] != nullptr));
    timed(c_, kClassElem, 0.0, by, [&] { return launch_lincomb(b_, ec_, a, c_->stream); });
  }

  void transcomb(const TransComb& t) {
    const double by = 16.0 * blk_ * ec_ * (1 + (t.C != nullptr) + (t.Z != nullptr));
    timed(c_, kClassElem, 0.0, by, [&] { return launch_transcomb(b_, ec_, t, c_->stream); });
  }

  // D(e) = C(e) + z Z(e) + g Z(e)^dag
  void antiherm(const View& D, long long id, const View* C, long long ic,
                const View& Z, long long iz, zc z, zc g) {
    TransComb t{};
    t.C = C ? C->at(ic) : nullptr; t.sC = C ? C->es : 0;
    t.Z = Z.at(iz); t.sZ = Z.es;
    t.D = D.w(id); t.sD = D.es;
    t.a = C ? kOne : kZero; t.z = z; t.g = g;
    transcomb(t);
  }

  void copy(const View& D, long long id, const View& S, long long is) {
    LinComb a{};
    a.src[0] = S.at(is); a.sSrc[0] = S.es; a.c[0] = kOne;
    a.D = D.w(id); a.sD = D.es;
    lincomb(a);
  }

  long long blk() const { return blk_; }
  int ec() const { return ec_; }

 private:
  qtx_rgf_ctx* c_;
  int b_, ec_;
  long long blk_;
  bool fp32_ = false;
};

// Operands of the recursion for one chunk.
struct Rhs {
  View Bd, Bu;             // B^s diag, upper (Bu may be empty)
  View Xd, Xu, Xl;         // outputs (Xl may be empty)
};

struct Core {
  int n;
  View U, L;               // U_i = su * U[i], L_i = sl * L[i]
  double su = 1.0, sl = 1.0;
  std::vector<Rhs> rhs;
  View XRd, XRu, XRl;
  View xR;                 // workspace [n] per energy
  View tS, tF, tP, tM, tR; // workspace, one block per energy
  View tG[2], tW[2], tY[2];
  InvWork inv;
  int* info;
};

// Forward and backward passes, given a callback that writes Mt_ii into tS.
template <class PrepDiag>
void run_core(Solver& s, const Core& k, PrepDiag prep_diag) {
  const int n = k.n;
  const int nr = (int)k.rhs.size();
  const zc su = rs(k.su), sl = rs(k.sl);

  // ---- forward pass ----------------------------------------------------
  prep_diag(0);
  s.inverse(k.tS, 0, k.xR, 0, k.inv, k.info, 1);
  if (nr == 2) {
    s.gemm('N', 'N', {Term{{k.xR, 0}, {k.rhs[0].Bd, 0}, nullptr, 0, k.tG[0], 0, kOne, kZero},
                      Term{{k.xR, 0}, {k.rhs[1].Bd, 0}, nullptr, 0, k.tG[1], 0, kOne, kZero}});
    s.gemm('N', 'C', {Term{{k.tG[0], 0}, {k.xR, 0}, nullptr, 0, k.rhs[0].Xd, 0, kOne, kZero},
                      Term{{k.tG[1], 0}, {k.xR, 0}, nullptr, 0, k.rhs[1].Xd, 0, kOne, kZero}});
  } else if (nr == 1) {
    s.gemm('N', 'N', {Term{{k.xR, 0}, {k.rhs[0].Bd, 0}, nullptr, 0, k.tG[0], 0, kOne, kZero}});
    s.gemm('N', 'C', {Term{{k.tG[0], 0}, {k.xR, 0}, nullptr, 0, k.rhs[0].Xd, 0, kOne, kZero}});
  }
  for (int i = 1; i < n; ++i) {
    // F = L_{i-1} x_{i-1};  Mt_ii - F U_{i-1}  -> inverse -> x_i
    s.gemm('N', 'N', {Term{{k.L, i - 1}, {k.xR, i - 1}, nullptr, 0, k.tF, 0, sl, kZero}});
    prep_diag(i);
    s.gemm('N', 'N', {Term{{k.tF, 0}, {k.U, i - 1}, &k.tS, 0, k.tS, 0, rs(-k.su), kOne}});
    s.inverse(k.tS, 0, k.xR, i, k.inv, k.info, i + 1);
    if (nr == 0) continue;
    // W = B_ii + L xs_{i-1} L^dag - y + y^dag;  xs_i = x_i W x_i^dag
    {
      Term t0{{k.L, i - 1}, {k.rhs[0].Xd, i - 1}, nullptr, 0, k.tG[0], 0, sl, kZero};
      if (nr == 2) {
        Term t1{{k.L, i - 1}, {k.rhs[1].Xd, i - 1}, nullptr, 0, k.tG[1], 0, sl, kZero};
        s.gemm('N', 'N', {t0, t1});
      } else {
        s.gemm('N', 'N', {t0});
      }
    }
    {
      Term t0{{k.tG[0], 0}, {k.L, i - 1}, &k.rhs[0].Bd, i, k.tW[0], 0, sl, kOne};
      if (nr == 2) {
        Term t1{{k.tG[1], 0}, {k.L, i - 1}, &k.rhs[1].Bd, i, k.tW[1], 0, sl, kOne};
        s.gemm('N', 'C', {t0, t1});
      } else {
        s.gemm('N', 'C', {t0});
      }
    }
    for (int r = 0; r < nr; ++r) {
      if (!k.rhs[r].Bu.ok()) continue;
      s.gemm('N', 'N', {Term{{k.tF, 0}, {k.rhs[r].Bu, i - 1}, nullptr, 0, k.tY[r], 0, kOne, kZero}});
      s.antiherm(k.tW[r], 0, &k.tW[r], 0, k.tY[r], 0, kMinus, kOne);
    }
    if (nr == 2) {
      s.gemm('N', 'N', {Term{{k.xR, i}, {k.tW[0], 0}, nullptr, 0, k.tG[0], 0, kOne, kZero},
                        Term{{k.xR, i}, {k.tW[1], 0}, nullptr, 0, k.tG[1], 0, kOne, kZero}});
      s.gemm('N', 'C', {Term{{k.tG[0], 0}, {k.xR, i}, nullptr, 0, k.rhs[0].Xd, i, kOne, kZero},
                        Term{{k.tG[1], 0}, {k.xR, i}, nullptr, 0, k.rhs[1].Xd, i, kOne, kZero}});
    } else {
      s.gemm('N', 'N', {Term{{k.xR, i}, {k.tW[0], 0}, nullptr, 0, k.tG[0], 0, kOne, kZero}});
      s.gemm('N', 'C', {Term{{k.tG[0], 0}, {k.xR, i}, nullptr, 0, k.rhs[0].Xd, i, kOne, kZero}});
    }
  }

  // ---- backward pass ---------------------------------------------------
  s.copy(k.XRd, n - 1, k.xR, n - 1);
  for (int i = n - 2; i >= 0; --i) {
    // P = x_i U_i,  M = X_{i+1} L_i
    s.gemm('N', 'N', {Term{{k.xR, i}, {k.U, i}, nullptr, 0, k.tP, 0, su, kZero},
                      Term{{k.XRd, i + 1}, {k.L, i}, nullptr, 0, k.tM, 0, sl, kZero}});
    // X_{i,i+1} = -P X_{i+1} (= -Q),  X_{i+1,i} = -M x_i
    s.gemm('N', 'N', {Term{{k.tP, 0}, {k.XRd, i + 1}, nullptr, 0, k.XRu, i, kMinus, kZero},
                      Term{{k.tM, 0}, {k.xR, i}, nullptr, 0, k.XRl, i, kMinus, kZero}});
    // R = Q L_i = -X_{i,i+1} L_i
    s.gemm('N', 'N', {Term{{k.XRu, i}, {k.L, i}, nullptr, 0, k.tR, 0, rs(-k.sl), kZero}});
    // X_i = x_i + R x_i
    s.gemm('N', 'N', {Term{{k.tR, 0}, {k.xR, i}, &k.xR, i, k.XRd, i, kOne, kOne}});
    if (nr == 0) continue;
    // T1 = P X^s_{i+1},  Z = R xs_i
    if (nr == 2) {
      s.gemm('N', 'N', {Term{{k.tP, 0}, {k.rhs[0].Xd, i + 1}, nullptr, 0, k.tG[0], 0, kOne, kZero},
                        Term{{k.tP, 0}, {k.rhs[1].Xd, i + 1}, nullptr, 0, k.tG[1], 0, kOne, kZero},
                        Term{{k.tR, 0}, {k.rhs[0].Xd, i}, nullptr, 0, k.tW[0], 0, kOne, kZero},
                        Term{{k.tR, 0}, {k.rhs[1].Xd, i}, nullptr, 0, k.tW[1], 0, kOne, kZero}});
      // X^s_{i,i+1} = -T1 - xs_i M^dag
      s.gemm('N', 'C', {Term{{k.rhs[0].Xd, i}, {k.tM, 0}, &k.tG[0], 0, k.rhs[0].Xu, i, kMinus, kMinus},
                        Term{{k.rhs[1].Xd, i}, {k.tM, 0}, &k.tG[1], 0, k.rhs[1].Xu, i, kMinus, kMinus}});
      // X^s_ii = xs_i + T1 P^dag (+ Z - Z^dag below)
      s.gemm('N', 'C', {Term{{k.tG[0], 0}, {k.tP, 0}, &k.rhs[0].Xd, i, k.rhs[0].Xd, i, kOne, kOne},
                        Term{{k.tG[1], 0}, {k.tP, 0}, &k.rhs[1].Xd, i, k.rhs[1].Xd, i, kOne, kOne}});
    } else {
      s.gemm('N', 'N', {Term{{k.tP, 0}, {k.rhs[0].Xd, i + 1}, nullptr, 0, k.tG[0], 0, kOne, kZero},
                        Term{{k.tR, 0}, {k.rhs[0].Xd, i}, nullptr, 0, k.tW[0], 0, kOne, kZero}});
      s.gemm('N', 'C', {Term{{k.rhs[0].Xd, i}, {k.tM, 0}, &k.tG[0], 0, k.rhs[0].Xu, i, kMinus, kMinus}});
      s.gemm('N', 'C', {Term{{k.tG[0], 0}, {k.tP, 0}, &k.rhs[0].Xd, i, k.rhs[0].Xd, i, kOne, kOne}});
    }
    for (int r = 0; r < nr; ++r) {
      const Rhs& h = k.rhs[r];
      s.antiherm(h.Xd, i, &h.Xd, i, k.tW[r], 0, kOne, kMinus);
      if (h.Bu.ok()) {
        // V = x_i B_{i,i+1};  X^s_{i,i+1} += V X_{i+1}^dag;  X^s_ii -= Y - Y^dag,
        // Y = V Q^dag = -V X_{i,i+1}^dag
        s.gemm('N', 'N', {Term{{k.xR, i}, {h.Bu, i}, nullptr, 0, k.tY[r], 0, kOne, kZero}});
        s.gemm('N', 'C', {Term{{k.tY[r], 0}, {k.XRd, i + 1}, &h.Xu, i, h.Xu, i, kOne, kOne}});
        s.gemm('N', 'C', {Term{{k.tY[r], 0}, {k.XRu, i}, nullptr, 0, k.tW[r], 0, kOne, kZero}});
        s.antiherm(h.Xd, i, &h.Xd, i, k.tW[r], 0, kOne, kMinus);
      }
      if (h.Xl.ok()) s.antiherm(h.Xl, i, nullptr, 0, h.Xu, i, kZero, kMinus);
    }
  }
}

// ------------------------------------------------------------ workspace ---

struct Carve {
  char* base;
  size_t cap;
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t o = (off + 255) & ~size_t(255);
    off = o + bytes;
    if (off > cap) throw Fail{QTX_ERR_NOMEM};   // never hand out memory past the workspace
    return o;
  }
};

bool bt_in_empty(const qtx_bt_in& t) { return !t.diag && !t.upper && !t.lower; }

struct Plan {
  int n, b, ne, nr;
  bool general_ul;     // U/L depend on energy (assembled per energy)
  bool need_hl;        // H.lower / V.lower absent for an operand used as N
  bool bt_rhs[2];
  bool is_w;
  size_t per_energy;   // workspace bytes per energy
  size_t fixed;        // energy-independent workspace bytes
};

size_t blocks_bytes(long long nblk, int b) { return (size_t)nblk * b * b * 16 + 256; }

Plan make_plan(const qtx_rgf_problem& p) {
  Plan q{};
  q.n = p.n_blocks; q.b = p.block_size; q.ne = p.n_energies;
  q.is_w = p.kind == QTX_KIND_W;
  q.nr = (p.XL.diag ? 1 : 0) + (p.XG.diag ? 1 : 0);
  const int n = q.n, b = q.b;
  int ri = 0;
  if (!q.is_w) {
    q.general_ul = (p.S.diag && (p.S.upper || p.S.lower)) || p.sigma_r.upper || p.sigma_r.lower;
    q.need_hl = (n > 1) && !p.H.lower;
    if (p.XL.diag) q.bt_rhs[ri++] = p.sigma_l.upper != nullptr && n > 1;
    if (p.XG.diag) q.bt_rhs[ri++] = p.sigma_g.upper != nullptr && n > 1;
  } else {
    q.general_ul = true;
    q.need_hl = false;
    for (int r = 0; r < q.nr; ++r) q.bt_rhs[r] = n > 1;
  }
  size_t pe = 0;
  pe += blocks_bytes(n, b);                    // x_i
  int ntmp = 5 + 2 * q.nr;
  for (int r = 0; r < q.nr; ++r) ntmp += q.bt_rhs[r] ? 1 : 0;
  pe += ntmp * blocks_bytes(1, b);
  if (q.general_ul) pe += 2 * blocks_bytes(std::max(n - 1, 0), b);
  pe += (size_t)b * kPanel * 16 * 2 + 1024 + (size_t)b * 8 + 512;   // inverse work
  pe += 64;                                                        // info, energy
  if (q.is_w) {
    pe += blocks_bytes(n, b);                                      // Mt diag
    pe += q.nr * (blocks_bytes(n, b) + blocks_bytes(std::max(n - 1, 0), b));  // B^s
    if (q.nr) pe += 4 * blocks_bytes(n, b);                        // V P^s blocks
  }
  q.per_energy = pe;
  q.fixed = q.need_hl ? blocks_bytes(std::max(n - 1, 0), b) : 0;
  q.fixed += 64 * 1024;      // alignment of the ~40 carved sub-buffers
  return q;
}

void ensure_ws(qtx_rgf_ctx* c, size_t bytes) {
  if (c->ws_bytes >= bytes) return;
  if (c->ws) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipFree(c->ws));
    c->ws = nullptr;
    c->ws_bytes = 0;
  }
  hipError_t e = hipMalloc(&c->ws, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    c->ws = nullptr;
    c->err = "workspace allocation of " + std::to_string(bytes) + " bytes failed";
    throw Fail{QTX_ERR_NOMEM};
  }
  c->ws_bytes = bytes;
}

size_t budget_now(qtx_rgf_ctx* c) {
  if (c->budget) return c->budget;
  size_t fr = 0, tot = 0;
  HIPCHK(c, hipMemGetInfo(&fr, &tot));
  size_t have = fr + c->ws_bytes;
  return (size_t)(0.9 * (double)have);
}

View in_view(const void* p, long long es, long long bs) {
  View v;
  v.p = (const double2*)p;
  v.es = es;
  v.bs = bs;
  return v;
}

// Validation of one problem; returns an error message or empty.
std::string validate(const qtx_rgf_problem& p) {
  if (p.kind != QTX_KIND_G && p.kind != QTX_KIND_W) return "unknown kind";
  if (p.precision != QTX_FP64 && p.precision != QTX_MIXED) return "unknown precision";
  if (p.n_blocks < 1 || p.block_size < 1 || p.n_energies < 1) return "n_blocks, block_size and n_energies must be >= 1";
  if (p.block_size > 1024) return "block_size above 1024 is not supported";
  if (p.flags != 0) return "flags must be 0";
  if (!p.XR.diag) return "XR.diag is required";
  if (p.n_blocks > 1 && (!p.XR.upper || !p.XR.lower)) return "XR.upper and XR.lower are required when n_blocks > 1";
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

// ---------------------------------------------------------------- W setup --

// Mt = I - trunc(V P^R), B^s = trunc(V P^s V^dag) for the chunk, written to
// the workspace views.  V lower = V upper^dag when absent; P^s lower =
// -(P^s upper)^dag (anti-Hermitian).
struct WOps {
  View Vd, Vu, Vl;        // Vl empty -> use Vu with op C
  View Prd, Pru, Prl;     // per energy
  View Psd[2], Psu[2];    // per energy
  View Ad, Au, Al;        // outputs (workspace)
  View Bd[2], Bu[2];      // outputs (workspace)
  View Tm1, T0, Tp1, Tp2; // scratch: (V P^s)_{i,i-1}, _{i,i}, _{i,i+1}, _{i,i+2}
};

void w_assemble(Solver& s, const WOps& w, int n, int nr) {
  const long long blk = s.blk();
  // identity into Ad
  for (int i = 0; i < n; ++i) {
    LinComb a{};
    a.idc0 = kOne;
    a.D = w.Ad.w(i); a.sD = w.Ad.es;
    s.lincomb(a);
  }
  (void)blk;
  const bool vl = w.Vl.ok();
  const char opVl = vl ? 'N' : 'C';            // V_{i+1,i} as stored operand
  const View& VL = vl ? w.Vl : w.Vu;
  // ---- Mt = I - trunc(V P^R) -------------------------------------------
  s.gemm('N', 'N', {Term{{w.Vd, 0}, {w.Prd, 0}, &w.Ad, 0, w.Ad, 0, kMinus, kOne}}, n);
  if (n > 1) {
    if (w.Pru.ok())   // Ad[i] -= V_{i,i-1} P_{i-1,i},  i >= 1
      s.gemm(opVl, 'N', {Term{{VL, 0}, {w.Pru, 0}, &w.Ad, 1, w.Ad, 1, kMinus, kOne}}, n - 1);
    if (w.Prl.ok())   // Ad[i] -= V_{i,i+1} P_{i+1,i},  i <= n-2
      s.gemm('N', 'N', {Term{{w.Vu, 0}, {w.Prl, 0}, &w.Ad, 0, w.Ad, 0, kMinus, kOne}}, n - 1);
    // Au[i] = -(V_ii P_{i,i+1} + V_{i,i+1} P_{i+1,i+1})
    if (w.Pru.ok()) {
      s.gemm('N', 'N', {Term{{w.Vd, 0}, {w.Pru, 0}, nullptr, 0, w.Au, 0, kMinus, kZero}}, n - 1);
      s.gemm('N', 'N', {Term{{w.Vu, 0}, {w.Prd, 1}, &w.Au, 0, w.Au, 0, kMinus, kOne}}, n - 1);
    } else {
      s.gemm('N', 'N', {Term{{w.Vu, 0}, {w.Prd, 1}, nullptr, 0, w.Au, 0, kMinus, kZero}}, n - 1);
    }
    // Al[i] = -(V_{i+1,i} P_ii + V_{i+1,i+1} P_{i+1,i})
    s.gemm(opVl, 'N', {Term{{VL, 0}, {w.Prd, 0}, nullptr, 0, w.Al, 0, kMinus, kZero}}, n - 1);
    if (w.Prl.ok())
      s.gemm('N', 'N', {Term{{w.Vd, 1}, {w.Prl, 0}, &w.Al, 0, w.Al, 0, kMinus, kOne}}, n - 1);
  }
  // ---- B^s = trunc(V P^s V^dag) ------------------------------------------
  for (int r = 0; r < nr; ++r) {
    const View& Pd = w.Psd[r];
    const View& Pu = w.Psu[r];
    const bool pu = Pu.ok() && n > 1;
    // T0[i] = V_ii P_ii (+ V_{i,i-1} P_{i-1,i} + V_{i,i+1} P_{i+1,i})
    s.gemm('N', 'N', {Term{{w.Vd, 0}, {Pd, 0}, nullptr, 0, w.T0, 0, kOne, kZero}}, n);
    if (n > 1) {
      if (pu) {
        s.gemm(opVl, 'N', {Term{{VL, 0}, {Pu, 0}, &w.T0, 1, w.T0, 1, kOne, kOne}}, n - 1);
        // P_{i+1,i} = -(P_{i,i+1})^dag
        s.gemm('N', 'C', {Term{{w.Vu, 0}, {Pu, 0}, &w.T0, 0, w.T0, 0, kMinus, kOne}}, n - 1);
      }
      // Tm1[i] = V_{i,i-1} P_{i-1,i-1} + V_ii P_{i,i-1},  i >= 1
      s.gemm(opVl, 'N', {Term{{VL, 0}, {Pd, 0}, nullptr, 0, w.Tm1, 1, kOne, kZero}}, n - 1);
      if (pu) s.gemm('N', 'C', {Term{{w.Vd, 1}, {Pu, 0}, &w.Tm1, 1, w.Tm1, 1, kMinus, kOne}}, n - 1);
      // Tp1[i] = V_ii P_{i,i+1} + V_{i,i+1} P_{i+1,i+1},  i <= n-2
      s.gemm('N', 'N', {Term{{w.Vu, 0}, {Pd, 1}, nullptr, 0, w.Tp1, 0, kOne, kZero}}, n - 1);
      if (pu) s.gemm('N', 'N', {Term{{w.Vd, 0}, {Pu, 0}, &w.Tp1, 0, w.Tp1, 0, kOne, kOne}}, n - 1);
      // Tp2[i] = V_{i,i+1} P_{i+1,i+2},  i <= n-3
      if (pu && n > 2) s.gemm('N', 'N', {Term{{w.Vu, 0}, {Pu, 1}, nullptr, 0, w.Tp2, 0, kOne, kZero}}, n - 2);
    }
    // B_ii = T0 V_ii^dag + Tm1 V_{i,i-1}^dag + Tp1 V_{i,i+1}^dag
    s.gemm('N', 'C', {Term{{w.T0, 0}, {w.Vd, 0}, nullptr, 0, w.Bd[r], 0, kOne, kZero}}, n);
    if (n > 1) {
      // V_{i,i-1}^dag: stored lower block adjoint, or (upper^dag)^dag = upper
      s.gemm('N', vl ? 'C' : 'N', {Term{{w.Tm1, 1}, {VL, 0}, &w.Bd[r], 1, w.Bd[r], 1, kOne, kOne}}, n - 1);
      s.gemm('N', 'C', {Term{{w.Tp1, 0}, {w.Vu, 0}, &w.Bd[r], 0, w.Bd[r], 0, kOne, kOne}}, n - 1);
      // B_{i,i+1} = T0 V_{i+1,i}^dag + Tp1 V_{i+1,i+1}^dag + Tp2 V_{i+1,i+2}^dag
      s.gemm('N', vl ? 'C' : 'N', {Term{{w.T0, 0}, {VL, 0}, nullptr, 0, w.Bu[r], 0, kOne, kZero}}, n - 1);
      s.gemm('N', 'C', {Term{{w.Tp1, 0}, {w.Vd, 1}, &w.Bu[r], 0, w.Bu[r], 0, kOne, kOne}}, n - 1);
      if (pu && n > 2)
        s.gemm('N', 'C', {Term{{w.Tp2, 0}, {w.Vu, 1}, &w.Bu[r], 0, w.Bu[r], 0, kOne, kOne}}, n - 2);
    }
  }
}

// ------------------------------------------------------------ one problem --

qtx_status solve_problem(qtx_rgf_ctx* c, qtx_rgf_problem& p) {
  p.status = QTX_OK;
  p.fail_energy = -1;
  p.fail_block = -1;
  const Plan q = make_plan(p);
  const int n = q.n, b = q.b, ne = q.ne, nr = q.nr;
  const long long blk = (long long)b * b;
  const size_t budget = budget_now(c);
  if (budget < q.fixed + q.per_energy) {
    c->err = "one energy needs " + std::to_string(q.fixed + q.per_energy) +
             " workspace bytes, budget is " + std::to_string(budget);
    throw Fail{QTX_ERR_NOMEM};
  }
  int ec = (int)std::min<size_t>((size_t)ne, (budget - q.fixed) / q.per_energy);
  ec = std::max(1, std::min(ec, 65535 / std::max(1, n)));
  ensure_ws(c, q.fixed + (size_t)ec * q.per_energy + 4096);

  Carve cv{(char*)c->ws, c->ws_bytes};
  auto blocks = [&](long long nblk_per_e) {
    View v;
    v.p = (const double2*)(cv.base + cv.take((size_t)ec * nblk_per_e * blk * 16));
    v.es = nblk_per_e * blk;
    v.bs = blk;
    return v;
  };
  Core k{};
  k.n = n;
  k.xR = blocks(n);
  k.tS = blocks(1); k.tF = blocks(1); k.tP = blocks(1); k.tM = blocks(1); k.tR = blocks(1);
  for (int r = 0; r < nr; ++r) {
    k.tG[r] = blocks(1);
    k.tW[r] = blocks(1);
    if (q.bt_rhs[r]) k.tY[r] = blocks(1);
  }
  View Uw, Lw;
  if (q.general_ul && n > 1) { Uw = blocks(n - 1); Lw = blocks(n - 1); }
  k.inv.panel = cv.base + cv.take((size_t)ec * b * kPanel * 16);
  k.inv.brow = cv.base + cv.take((size_t)ec * b * kPanel * 16);
  k.inv.perm = (int*)(cv.base + cv.take((size_t)ec * b * 4));
  k.inv.used = (int*)(cv.base + cv.take((size_t)ec * b * 4));
  int* d_info = (int*)(cv.base + cv.take((size_t)ec * 4));
  double* d_E = (double*)(cv.base + cv.take((size_t)ec * 8));
  k.info = d_info;
  View Hl;
  if (q.need_hl) {
    Hl.p = (const double2*)(cv.base + cv.take((size_t)(n - 1) * blk * 16));
    Hl.es = 0;
    Hl.bs = blk;
  }
  WOps w{};
  if (q.is_w) {
    w.Ad = blocks(n);
    if (n > 1) { w.Au = Uw; w.Al = Lw; }
    for (int r = 0; r < nr; ++r) {
      w.Bd[r] = blocks(n);
      if (n > 1) w.Bu[r] = blocks(n - 1);
    }
    if (nr) { w.Tm1 = blocks(n); w.T0 = blocks(n); w.Tp1 = blocks(n); w.Tp2 = blocks(n); }
  }

  // H lower = H upper^dag when absent (energy independent, built once)
  if (q.need_hl) {
    Solver s1(c, b, 1);
    for (int i = 0; i < n - 1; ++i) {
      TransComb t{};
      t.Z = (const double2*)p.H.upper + i * blk;
      t.D = Hl.w(i);
      t.a = kZero; t.z = kZero; t.g = kOne;
      s1.transcomb(t);
    }
  }

  std::vector<int> h_info(ec);
  for (int e0 = 0; e0 < ne; e0 += ec) {
    const int ecur = std::min(ec, ne - e0);
    Solver sc(c, b, ecur);
    HIPCHK(c, hipMemsetAsync(d_info, 0, sizeof(int) * ecur, c->stream));
    // outputs
    auto outv = [&](void* ptr, long long per_e) {
      View v;
      if (!ptr) return v;
      v.p = (const double2*)ptr + (long long)e0 * per_e * blk;
      v.es = per_e * blk;
      v.bs = blk;
      return v;
    };
    auto inv_ = [&](const void* ptr, long long per_e) {
      View v;
      if (!ptr) return v;
      v.p = (const double2*)ptr + (long long)e0 * per_e * blk;
      v.es = per_e * blk;
      v.bs = blk;
      return v;
    };
    k.XRd = outv(p.XR.diag, n);
    k.XRu = outv(p.XR.upper, n - 1);
    k.XRl = outv(p.XR.lower, n - 1);
    k.rhs.clear();
    const qtx_bt_out* outs[2] = {&p.XL, &p.XG};
    int r = 0;
    for (int t = 0; t < 2; ++t) {
      if (!outs[t]->diag) continue;
      Rhs h;
      h.Xd = outv(outs[t]->diag, n);
      if (n > 1) {
        h.Xu = outv(outs[t]->upper, n - 1);
        h.Xl = outv(outs[t]->lower, n - 1);
      }
      if (!q.is_w) {
        const qtx_bt_in& B = t == 0 ? p.sigma_l : p.sigma_g;
        h.Bd = inv_(B.diag, n);
        if (n > 1 && B.upper) h.Bu = inv_(B.upper, n - 1);
      } else {
        h.Bd = w.Bd[r];
        if (n > 1) h.Bu = w.Bu[r];
      }
      k.rhs.push_back(h);
      ++r;
    }

    if (!q.is_w) {
      HIPCHK(c, hipMemcpyAsync(d_E, p.energies + e0, sizeof(double) * ecur, hipMemcpyHostToDevice, c->stream));
      const View Hd = in_view(p.H.diag, 0, blk);
      const View Hu = in_view(p.H.upper, 0, blk);
      const View HL = p.H.lower ? in_view(p.H.lower, 0, blk) : Hl;
      const View Sd = in_view(p.S.diag, 0, blk);
      const View SRd = inv_(p.sigma_r.diag, n);
      if (q.general_ul && n > 1) {
        const View Su = in_view(p.S.upper, 0, blk), Sl = in_view(p.S.lower, 0, blk);
        const View SRu = inv_(p.sigma_r.upper, n - 1), SRl = inv_(p.sigma_r.lower, n - 1);
        for (int i = 0; i < n - 1; ++i) {
          LinComb a{};
          a.E = d_E;
          a.src[0] = Hu.at(i); a.sSrc[0] = 0; a.c[0] = kMinus;
          if (Su.ok()) { a.src[1] = Su.at(i); a.sSrc[1] = 0; a.d[1] = kOne; }
          if (SRu.ok()) { a.src[2] = SRu.at(i); a.sSrc[2] = SRu.es; a.c[2] = kMinus; }
          a.D = Uw.w(i); a.sD = Uw.es;
          sc.lincomb(a);
          LinComb l{};
          l.E = d_E;
          l.src[0] = HL.at(i); l.sSrc[0] = 0; l.c[0] = kMinus;
          if (Sl.ok()) { l.src[1] = Sl.at(i); l.sSrc[1] = 0; l.d[1] = kOne; }
          if (SRl.ok()) { l.src[2] = SRl.at(i); l.sSrc[2] = SRl.es; l.c[2] = kMinus; }
          l.D = Lw.w(i); l.sD = Lw.es;
          sc.lincomb(l);
        }
        k.U = Uw; k.L = Lw; k.su = 1.0; k.sl = 1.0;
      } else {
        k.U = Hu; k.L = HL; k.su = -1.0; k.sl = -1.0;
      }
      sc.set_fp32_products(p.precision == QTX_MIXED);
      run_core(sc, k, [&](int i) {
        LinComb a{};
        a.E = d_E;
        if (Sd.ok()) { a.src[0] = Sd.at(i); a.sSrc[0] = 0; a.d[0] = kOne; }
        else a.idc1 = kOne;
        a.src[1] = Hd.at(i); a.sSrc[1] = 0; a.c[1] = kMinus;
        a.src[2] = SRd.at(i); a.sSrc[2] = SRd.es; a.c[2] = kMinus;
        a.D = k.tS.w(0); a.sD = k.tS.es;
        sc.lincomb(a);
      });
    } else {
      w.Vd = in_view(p.V.diag, 0, blk);
      w.Vu = in_view(p.V.upper, 0, blk);
      w.Vl = in_view(p.V.lower, 0, blk);
      w.Prd = inv_(p.P_r.diag, n);
      w.Pru = n > 1 ? inv_(p.P_r.upper, n - 1) : View();
      w.Prl = n > 1 ? inv_(p.P_r.lower, n - 1) : View();
      const qtx_bt_in* Ps[2] = {&p.P_l, &p.P_g};
      int rr = 0;
      for (int t = 0; t < 2; ++t) {
        if (!outs[t]->diag) continue;
        w.Psd[rr] = inv_(Ps[t]->diag, n);
        w.Psu[rr] = n > 1 ? inv_(Ps[t]->upper, n - 1) : View();
        ++rr;
      }
      w_assemble(sc, w, n, nr);
      k.U = w.Au; k.L = w.Al; k.su = 1.0; k.sl = 1.0;
      sc.set_fp32_products(p.precision == QTX_MIXED);
      run_core(sc, k, [&](int i) { sc.copy(k.tS, 0, w.Ad, i); });
      sc.set_fp32_products(false);
      if (p.WR_diag) {
        // W^R_ii = X_ii V_ii + X_{i,i-1} V_{i-1,i} + X_{i,i+1} V_{i+1,i}
        const View WR = outv(p.WR_diag, n);
        sc.gemm('N', 'N', {Term{{k.XRd, 0}, {w.Vd, 0}, nullptr, 0, WR, 0, kOne, kZero}}, n);
        if (n > 1) {
          sc.gemm('N', 'N', {Term{{k.XRl, 0}, {w.Vu, 0}, &WR, 1, WR, 1, kOne, kOne}}, n - 1);
          const bool vl = w.Vl.ok();
          sc.gemm('N', vl ? 'N' : 'C', {Term{{k.XRu, 0}, {vl ? w.Vl : w.Vu, 0}, &WR, 0, WR, 0, kOne, kOne}}, n - 1);
        }
      }
    }

    HIPCHK(c, hipMemcpyAsync(h_info.data(), d_info, sizeof(int) * ecur, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    flush_stats(c);
    for (int e = 0; e < ecur; ++e) {
      if (h_info[e] != 0 && p.status == QTX_OK) {
        p.status = h_info[e] > 0 ? QTX_ERR_SINGULAR : QTX_ERR_NOT_FINITE;
        p.fail_energy = e0 + e;
        p.fail_block = std::abs(h_info[e]) - 1;
      }
    }
  }
  return p.status == QTX_OK ? QTX_OK : QTX_ERR_PROBLEM;
}

struct BusyGuard {
  qtx_rgf_ctx* c;
  explicit BusyGuard(qtx_rgf_ctx* c_) : c(c_) { c->busy = true; }
  ~BusyGuard() { c->busy = false; }
};

}  // namespace

// ==================================================================== ABI ==

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

qtx_status qtx_rgf_create(qtx_rgf_ctx** out, int device, uint64_t budget,
                          void* stream, uint32_t flags) {
  if (!out) return QTX_ERR_INVALID_ARG;
  *out = nullptr;
  if (flags & ~QTX_FLAG_PROFILE) return QTX_ERR_INVALID_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return device < 0 ? QTX_ERR_INVALID_ARG : QTX_ERR_HIP;
  }
  qtx_rgf_ctx* c = new (std::nothrow) qtx_rgf_ctx();
  if (!c) return QTX_ERR_NOMEM;
  c->device = device;
  c->budget = budget;
  c->flags = flags;
  if (hipSetDevice(device) != hipSuccess) { delete c; return QTX_ERR_HIP; }
  if (stream) {
    c->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return QTX_ERR_HIP;
    }
    c->own_stream = true;
  }
  *out = c;
  return QTX_OK;
}

qtx_status qtx_rgf_destroy(qtx_rgf_ctx* c) {
  if (!c) return QTX_ERR_INVALID_ARG;
  if (c->busy) return QTX_ERR_BUSY;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (auto& p : c->pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
  for (auto e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->ws) (void)hipFree(c->ws);
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
    std::string m = validate(probs[i]);
    if (!m.empty()) { c->err = "problem " + std::to_string(i) + ": " + m; return QTX_ERR_INVALID_ARG; }
  }
  BusyGuard g(c);
  qtx_status worst = QTX_OK;
  try {
    if (hipSetDevice(c->device) != hipSuccess) { c->err = "hipSetDevice failed"; return QTX_ERR_HIP; }
    for (int i = 0; i < np; ++i) {
      qtx_status st = solve_problem(c, probs[i]);
      if (st != QTX_OK) worst = st;
    }
  } catch (const Fail& f) {
    (void)hipStreamSynchronize(c->stream);
    flush_stats(c);
    return f.st;
  } catch (...) {
    c->err = "internal error";
    return QTX_ERR_HIP;
  }
  return worst;
}

double qtx_rgf_flops_per_energy(int32_t kind, int32_t n, int32_t b, int32_t n_rhs,
                                int32_t bt_rhs, int32_t want_wr) {
  if (n < 1 || b < 1 || n_rhs < 0) return 0.0;
  const double g = 8.0 * (double)b * b * b;
  const int per_fwd = 4 + (bt_rhs ? 1 : 0);
  const int per_bwd = 4 + (bt_rhs ? 3 : 0);
  double cnt = 1 + 2.0 * n_rhs + (n - 1.0) * (3 + per_fwd * n_rhs) + (n - 1.0) * (6 + per_bwd * n_rhs);
  if (kind == QTX_KIND_W) {
    // W assembly with block-tridiagonal P^R and P^s (see the flop model in
    // the tests' oracle): products needed for trunc(V P^R) and the diagonal
    // and upper blocks of trunc(V P^s V^dag).
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

qtx_status qtx_rgf_kernel_stats(qtx_rgf_ctx* c, int32_t cls, int64_t* launches,
                                double* ms, double* flops, double* bytes) {
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
                    int32_t k, double ar, double ai, const void* A, int64_t lda,
                    int64_t sA, const void* B, int64_t ldb, int64_t sB,
                    double br, double bi, const void* C, int64_t ldc, int64_t sC,
                    void* D, int64_t ldd, int64_t sD, int32_t batch) {
  if (!c) return QTX_ERR_INVALID_ARG;
  if ((opa != 'N' && opa != 'C') || (opb != 'N' && opb != 'C') || m < 0 || n < 0 ||
      k < 0 || batch < 0 || batch > 65535 || !A || !B || !D || (!C && (br != 0.0 || bi != 0.0)))
    return QTX_ERR_INVALID_ARG;
  const int64_t colsA = opa == 'N' ? k : m;
  const int64_t colsB = opb == 'N' ? n : k;
  if (lda < std::max<int64_t>(1, colsA) || ldb < std::max<int64_t>(1, colsB) ||
      ldd < std::max<int64_t>(1, n) || (C && ldc < std::max<int64_t>(1, n)))
    return QTX_ERR_INVALID_ARG;
  if (m == 0 || n == 0 || batch == 0) return QTX_OK;
  try {
    HIPCHK(c, hipSetDevice(c->device));
    GemmArgs g{};
    g.M = m; g.N = n; g.K = k;
    g.lda = lda; g.ldb = ldb; g.ldc = C ? ldc : ldd; g.ldd = ldd;
    g.batch = batch; g.batch2 = 1; g.ngroups = 1;
    g.g[0].A = A; g.g[0].sA = sA;
    g.g[0].B = B; g.g[0].sB = sB;
    g.g[0].C = C; g.g[0].sC = sC;
    g.g[0].D = D; g.g[0].sD = sD;
    g.g[0].alpha = zc{ar, ai};
    g.g[0].beta = C ? zc{br, bi} : kZero;
    const double fl = 8.0 * m * n * (double)k * batch;
    const double by = 16.0 * ((double)m * k + (double)k * n + (C ? 2.0 : 1.0) * m * n) * batch;
    timed(c, fp32 ? kClassCgemm : kClassZgemm, fl, by, [&] {
      return fp32 ? launch_cgemm(opa, opb, g, c->stream) : launch_zgemm(opa, opb, g, c->stream);
    });
    HIPCHK(c, hipStreamSynchronize(c->stream));
    flush_stats(c);
  } catch (const Fail& f) {
    return f.st;
  }
  return QTX_OK;
}
}  // namespace

extern "C" {

qtx_status qtx_rgf_zgemm(qtx_rgf_ctx* c, char opa, char opb, int32_t m, int32_t n,
                         int32_t k, double ar, double ai, const void* A, int64_t lda,
                         int64_t sA, const void* B, int64_t ldb, int64_t sB,
                         double br, double bi, const void* C, int64_t ldc, int64_t sC,
                         void* D, int64_t ldd, int64_t sD, int32_t batch) {
  return gemm_abi(false, c, opa, opb, m, n, k, ar, ai, A, lda, sA, B, ldb, sB, br, bi,
                  C, ldc, sC, D, ldd, sD, batch);
}

qtx_status qtx_rgf_cgemm(qtx_rgf_ctx* c, char opa, char opb, int32_t m, int32_t n,
                         int32_t k, double ar, double ai, const void* A, int64_t lda,
                         int64_t sA, const void* B, int64_t ldb, int64_t sB,
                         double br, double bi, const void* C, int64_t ldc, int64_t sC,
                         void* D, int64_t ldd, int64_t sD, int32_t batch) {
  return gemm_abi(true, c, opa, opb, m, n, k, ar, ai, A, lda, sA, B, ldb, sB, br, bi,
                  C, ldc, sC, D, ldd, sD, batch);
}

qtx_status qtx_rgf_zinv(qtx_rgf_ctx* c, int32_t b, void* A, void* X, int32_t* info,
                        int32_t batch) {
  if (!c || b < 1 || b > 1024 || !A || !X || batch < 0 || batch > 65535 || A == X)
    return QTX_ERR_INVALID_ARG;
  if (batch == 0) return QTX_OK;
  void* work = nullptr;
  try {
    HIPCHK(c, hipSetDevice(c->device));
    const size_t pan = (size_t)batch * b * kPanel * 16;
    const size_t ints = (size_t)batch * b * 4;
    HIPCHK(c, hipMalloc(&work, 2 * pan + 2 * ints + 1024));
    InvWork w{};
    w.panel = work;
    w.brow = (char*)work + pan;
    w.perm = (int*)((char*)work + 2 * pan);
    w.used = (int*)((char*)work + 2 * pan + ints);
    if (info) HIPCHK(c, hipMemsetAsync(info, 0, sizeof(int) * batch, c->stream));
    const double fl = 8.0 * (double)b * b * b * batch;
    timed(c, kClassInv, fl, 32.0 * b * b * batch, [&] {
      return launch_zinv(b, A, (long long)b * b, X, (long long)b * b, batch, w, info, 0, c->stream);
    });
    HIPCHK(c, hipStreamSynchronize(c->stream));
    flush_stats(c);
    HIPCHK(c, hipFree(work));
  } catch (const Fail& f) {
    if (work) (void)hipFree(work);
    return f.st;
  }
  return QTX_OK;
}

}  // extern "C"
