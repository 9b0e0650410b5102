// The RGF recursion of one lane as a list of block operations
// (arXiv 2508.19138, Sec. 3.2.3, Eqs. forward-pass / backward-pass; system
// assembly of Sec. 3.2.2 and Table "quantities").
//
// Notation: x_i = x^R_i (left-connected), xs_i = x^s_i, X_i = X^R_i,
// U_i = Mt_{i,i+1}, L_i = Mt_{i+1,i}.  The right-hand sides are
// anti-Hermitian, so each of  y - y^dag,  Y - Y^dag  and  Z - Z^dag  needs a
// single product, and the lower blocks of X^s are -upper^dagger.
#include "emit.h"

#include <algorithm>
#include <initializer_list>

namespace qtx {
namespace {

const zc kOne{1.0, 0.0}, kZero{0.0, 0.0}, kMinus{-1.0, 0.0};
inline zc rs(double v) { return zc{v, 0.0}; }

// A block-indexed operand: block i of energy e (relative to the view's
// base) starts at p + e * es + i * bs (complex elements).
struct View {
  const double2* p = nullptr;
  long long es = 0, bs = 0;
  bool ok() const { return p != nullptr; }
  const double2* at(long long i) const { return p + i * bs; }
  double2* w(long long i) const { return const_cast<double2*>(p + i * bs); }
};

struct Opnd {
  View v;
  long long i;
};

struct Term {            // D = alpha * A B + beta * C, batched over energies
  Opnd A, B;
  const View* C;         // null = no C
  long long ic;
  View D;
  long long id;
  zc alpha, beta;
};

class Emitter {
 public:
  Emitter(Lane& L, Tuner& T, hipStream_t s, int b, int ec)
      : L_(L), T_(T), s_(s), b_(b), ec_(ec), blk_((long long)b * b) {}
  void set_fp32(bool on) { fp32_ = on; }

  // One operation: the terms are independent products with the same
  // operand ops; `nb2` consecutive blocks (each view's bs) form a second
  // batch index.
  void gemm(char opa, char opb, std::initializer_list<Term> terms, int nb2 = 1) {
    Op o;
    o.k = OpK::Gemm;
    o.opa = opa; o.opb = opb; o.fp32 = fp32_;
    o.cfg = T_.cfg(b_, b_, b_, fp32_, s_);
    o.first = (int)L_.gd.size();
    for (const Term& t : terms) {
      GemmDesc g{};
      g.A = t.A.v.at(t.A.i); g.sA = t.A.v.es; g.tA = t.A.v.bs;
      g.B = t.B.v.at(t.B.i); g.sB = t.B.v.es; g.tB = t.B.v.bs;
      if (t.C) { g.C = t.C->at(t.ic); g.sC = t.C->es; g.tC = t.C->bs; }
      g.D = t.D.w(t.id); g.sD = t.D.es; g.tD = t.D.bs;
      g.lda = g.ldb = g.ldc = g.ldd = b_;
      g.alpha = t.alpha;
      g.beta = t.C ? t.beta : kZero;
      g.M = g.N = g.K = b_;
      g.batch = ec_;
      g.batch2 = nb2;
      L_.gd.push_back(g);
      o.flops += 8.0 * blk_ * b_ * (double)ec_ * nb2;
      o.bytes += 16.0 * blk_ * (t.C ? 4.0 : 3.0) * ec_ * nb2;
    }
    o.count = (int)L_.gd.size() - o.first;
    L_.ops.push_back(o);
  }

  void inverse(const View& S, long long is, const View& X, long long ix, void* panel,
               void* brow, void* spanel, void* sbrow, int* perm, int* used, int* info,
               int code, bool reset) {
    Op o;
    o.k = OpK::Inv;
    o.first = (int)L_.id.size();
    InvDesc d{};
    d.S = S.w(is); d.sS = S.es;
    d.X = X.w(ix); d.sX = X.es;
    d.panel = panel; d.brow = brow; d.spanel = spanel; d.sbrow = sbrow;
    d.perm = perm; d.used = used;
    d.info = info; d.code = code; d.reset_info = reset ? 1 : 0;
    d.b = b_; d.batch = ec_;
    L_.id.push_back(d);
    o.count = 1;
    o.flops = 8.0 * blk_ * b_ * ec_;
    L_.ops.push_back(o);
  }

  void lincomb(LinCombDesc a) {
    Op o;
    o.k = OpK::Lin;
    o.first = (int)L_.ld.size();
    a.b = b_;
    a.batch = ec_;
    L_.ld.push_back(a);
    o.count = 1;
    o.bytes = 16.0 * blk_ * ec_ * (1 + (a.src[0] != nullptr) + (a.src[1] != nullptr) + (a.src[2] != nullptr));
    L_.ops.push_back(o);
  }

  // D(e) = C(e) + z Z(e) + g Z(e)^dag, for up to two independent targets.
  void antiherm2(int count, const View* D, const long long* id, const View* const* C,
                 const long long* ic, const View* Z, const long long* iz, zc z, zc g) {
    Op o;
    o.k = OpK::Trans;
    o.first = (int)L_.td.size();
    for (int q = 0; q < count; ++q) {
      TransDesc t{};
      t.C = C[q] ? C[q]->at(ic[q]) : nullptr; t.sC = C[q] ? C[q]->es : 0;
      t.Z = Z[q].at(iz[q]); t.sZ = Z[q].es;
      t.D = D[q].w(id[q]); t.sD = D[q].es;
      t.a = C[q] ? kOne : kZero; t.z = z; t.g = g;
      t.b = b_; t.batch = ec_;
      L_.td.push_back(t);
      o.bytes += 16.0 * blk_ * ec_ * (2 + (C[q] != nullptr));
    }
    o.count = count;
    L_.ops.push_back(o);
  }
  void antiherm(const View& D, long long id, const View* C, long long ic,
                const View& Z, long long iz, zc z, zc g) {
    const View* Cs[1] = {C};
    antiherm2(1, &D, &id, Cs, &ic, &Z, &iz, z, g);
  }

  void copy(const View& D, long long id, const View& S, long long is) {
    LinCombDesc a{};
    a.src[0] = S.at(is); a.sSrc[0] = S.es; a.c[0] = kOne;
    a.D = D.w(id); a.sD = D.es;
    lincomb(a);
  }

  long long blk() const { return blk_; }

 private:
  Lane& L_;
  Tuner& T_;
  hipStream_t s_;
  int b_, ec_;
  long long blk_;
  bool fp32_ = false;
};

struct Rhs {
  View Bd, Bu;             // B^s diag, upper (Bu may be empty)
  View Xd, Xu, Xl;         // outputs (Xl may be empty)
};

struct Core {
  int n = 0;
  View U, L;               // U_i = su * U[i], L_i = sl * L[i]
  double su = 1.0, sl = 1.0;
  // Optional stored adjoints: U_i = (suh * Uh[i])^dag, L_i = (slh * Lh[i])^dag.
  // With them every product with U or L reads its other operand in the
  // orientation the matrix cores handle fastest (see Src below).
  View Uh, Lh;
  double suh = 1.0, slh = 1.0;
  std::vector<Rhs> rhs;
  View XRd, XRu, XRl;
  View xR;                 // workspace [n] per energy
  View tS, tF, tP, tM, tR; // workspace, one block per energy
  View tG[2], tW[2], tY[2];
  void *panel = nullptr, *brow = nullptr, *spanel = nullptr, *sbrow = nullptr;
  int *perm = nullptr, *used = nullptr, *info = nullptr;
};

// One product operand: value = sg * op(v[i]), op = 'N' (as stored) or 'C'
// (adjoint of the stored block).  Products whose operands are both stored
// as-is run markedly slower on the matrix-core kernel than products with one
// adjoint operand (measured on gfx950), so operands that have an exact
// adjoint relation are read through it: anti-Hermitian blocks
// (B^s, x^s_i, X^s_i and the bracket W of the forward step, B = -B^dag) and
// the couplings U, L of a Hermitian H (U = -H_u = (-H_l)^dag, L = (-H_u)^dag).
struct Src {
  View v;
  long long i;
  char op;
  double sg;
};
inline Src SN(const View& v, long long i, double sg = 1.0) { return Src{v, i, 'N', sg}; }
inline Src SC(const View& v, long long i, double sg = 1.0) { return Src{v, i, 'C', sg}; }
// anti-Hermitian block as an operand: B = -B^dag
inline Src SAH(const View& v, long long i) { return Src{v, i, 'C', -1.0}; }

struct Prod {             // D = alpha * a b + beta * C
  View D;
  long long id;
  Src a, b;
  const View* C;
  long long ic;
  double alpha, beta;
};

// Emit independent products; those sharing operand ops share one operation.
void prods(Emitter& s, std::initializer_list<Prod> ps) {
  const char combos[4][2] = {{'N', 'N'}, {'N', 'C'}, {'C', 'N'}, {'C', 'C'}};
  for (const auto& cb : combos) {
    Term t[4];
    int cnt = 0;
    for (const Prod& p : ps) {
      if (p.a.op != cb[0] || p.b.op != cb[1]) continue;
      t[cnt++] = Term{{p.a.v, p.a.i}, {p.b.v, p.b.i}, p.C, p.ic, p.D, p.id,
                      rs(p.alpha * p.a.sg * p.b.sg), rs(p.beta)};
    }
    if (cnt == 1) s.gemm(cb[0], cb[1], {t[0]});
    else if (cnt == 2) s.gemm(cb[0], cb[1], {t[0], t[1]});
    else if (cnt == 3) s.gemm(cb[0], cb[1], {t[0], t[1], t[2]});
    else if (cnt == 4) s.gemm(cb[0], cb[1], {t[0], t[1], t[2], t[3]});
  }
}

// Forward and backward passes, given a callback that writes Mt_ii into tS.
template <class PrepDiag>
void run_core(Emitter& s, const Core& k, PrepDiag prep_diag) {
  const int n = k.n;
  const int nr = (int)k.rhs.size();
  const bool uh = k.Uh.ok(), lh = k.Lh.ok();
  auto Ur = [&](long long i) { return uh ? SC(k.Uh, i, k.suh) : SN(k.U, i, k.su); };   // U_i
  auto Lr = [&](long long i) { return lh ? SC(k.Lh, i, k.slh) : SN(k.L, i, k.sl); };   // L_i
  auto LHr = [&](long long i) { return lh ? SN(k.Lh, i, k.slh) : SC(k.L, i, k.sl); };  // L_i^dag
  auto inv = [&](int i) {
    s.inverse(k.tS, 0, k.xR, i, k.panel, k.brow, k.spanel, k.sbrow, k.perm, k.used, k.info,
              i + 1, i == 0);
  };
  const View* none = nullptr;

  // ---- forward pass ----------------------------------------------------
  prep_diag(0);
  inv(0);
  if (nr >= 1) {
    // x^s_0 = x_0 B_00 x_0^dag
    if (nr == 2)
      prods(s, {Prod{k.tG[0], 0, SN(k.xR, 0), SAH(k.rhs[0].Bd, 0), none, 0, 1.0, 0.0},
                Prod{k.tG[1], 0, SN(k.xR, 0), SAH(k.rhs[1].Bd, 0), none, 0, 1.0, 0.0}});
    else
      prods(s, {Prod{k.tG[0], 0, SN(k.xR, 0), SAH(k.rhs[0].Bd, 0), none, 0, 1.0, 0.0}});
    if (nr == 2)
      prods(s, {Prod{k.rhs[0].Xd, 0, SN(k.tG[0], 0), SC(k.xR, 0), none, 0, 1.0, 0.0},
                Prod{k.rhs[1].Xd, 0, SN(k.tG[1], 0), SC(k.xR, 0), none, 0, 1.0, 0.0}});
    else
      prods(s, {Prod{k.rhs[0].Xd, 0, SN(k.tG[0], 0), SC(k.xR, 0), none, 0, 1.0, 0.0}});
  }
  for (int i = 1; i < n; ++i) {
    // F = L_{i-1} x_{i-1};  Mt_ii - F U_{i-1}  -> inverse -> x_i
    prods(s, {Prod{k.tF, 0, Lr(i - 1), SN(k.xR, i - 1), none, 0, 1.0, 0.0}});
    prep_diag(i);
    prods(s, {Prod{k.tS, 0, SN(k.tF, 0), Ur(i - 1), &k.tS, 0, -1.0, 1.0}});
    inv(i);
    if (nr == 0) continue;
    // W = B_ii + L x^s_{i-1} L^dag - y + y^dag;  x^s_i = x_i W x_i^dag
    if (nr == 2) {
      prods(s, {Prod{k.tG[0], 0, Lr(i - 1), SAH(k.rhs[0].Xd, i - 1), none, 0, 1.0, 0.0},
                Prod{k.tG[1], 0, Lr(i - 1), SAH(k.rhs[1].Xd, i - 1), none, 0, 1.0, 0.0}});
      prods(s, {Prod{k.tW[0], 0, SN(k.tG[0], 0), LHr(i - 1), &k.rhs[0].Bd, i, 1.0, 1.0},
                Prod{k.tW[1], 0, SN(k.tG[1], 0), LHr(i - 1), &k.rhs[1].Bd, i, 1.0, 1.0}});
    } else {
      prods(s, {Prod{k.tG[0], 0, Lr(i - 1), SAH(k.rhs[0].Xd, i - 1), none, 0, 1.0, 0.0}});
      prods(s, {Prod{k.tW[0], 0, SN(k.tG[0], 0), LHr(i - 1), &k.rhs[0].Bd, i, 1.0, 1.0}});
    }
    for (int r = 0; r < nr; ++r) {
      if (!k.rhs[r].Bu.ok()) continue;
      prods(s, {Prod{k.tY[r], 0, SN(k.tF, 0), SN(k.rhs[r].Bu, i - 1), none, 0, 1.0, 0.0}});
      s.antiherm(k.tW[r], 0, &k.tW[r], 0, k.tY[r], 0, kMinus, kOne);
    }
    if (nr == 2) {
      prods(s, {Prod{k.tG[0], 0, SN(k.xR, i), SAH(k.tW[0], 0), none, 0, 1.0, 0.0},
                Prod{k.tG[1], 0, SN(k.xR, i), SAH(k.tW[1], 0), none, 0, 1.0, 0.0}});
      prods(s, {Prod{k.rhs[0].Xd, i, SN(k.tG[0], 0), SC(k.xR, i), none, 0, 1.0, 0.0},
                Prod{k.rhs[1].Xd, i, SN(k.tG[1], 0), SC(k.xR, i), none, 0, 1.0, 0.0}});
    } else {
      prods(s, {Prod{k.tG[0], 0, SN(k.xR, i), SAH(k.tW[0], 0), none, 0, 1.0, 0.0}});
      prods(s, {Prod{k.rhs[0].Xd, i, SN(k.tG[0], 0), SC(k.xR, i), none, 0, 1.0, 0.0}});
    }
  }

  // ---- backward pass ---------------------------------------------------
  s.copy(k.XRd, n - 1, k.xR, n - 1);
  for (int i = n - 2; i >= 0; --i) {
    // P = x_i U_i,  M = X_{i+1} L_i
    prods(s, {Prod{k.tP, 0, SN(k.xR, i), Ur(i), none, 0, 1.0, 0.0},
              Prod{k.tM, 0, SN(k.XRd, i + 1), Lr(i), none, 0, 1.0, 0.0}});
    // X_{i,i+1} = -P X_{i+1} (= -Q),  X_{i+1,i} = -M x_i
    prods(s, {Prod{k.XRu, i, SN(k.tP, 0), SN(k.XRd, i + 1), none, 0, -1.0, 0.0},
              Prod{k.XRl, i, SN(k.tM, 0), SN(k.xR, i), none, 0, -1.0, 0.0}});
    // R = Q L_i = -X_{i,i+1} L_i
    prods(s, {Prod{k.tR, 0, SN(k.XRu, i), Lr(i), none, 0, -1.0, 0.0}});
    // X_i = x_i + R x_i
    prods(s, {Prod{k.XRd, i, SN(k.tR, 0), SN(k.xR, i), &k.xR, i, 1.0, 1.0}});
    if (nr == 0) continue;
    if (nr == 2) {
      // T1 = P X^s_{i+1},  Z = R x^s_i
      prods(s, {Prod{k.tG[0], 0, SN(k.tP, 0), SAH(k.rhs[0].Xd, i + 1), none, 0, 1.0, 0.0},
                Prod{k.tG[1], 0, SN(k.tP, 0), SAH(k.rhs[1].Xd, i + 1), none, 0, 1.0, 0.0},
                Prod{k.tW[0], 0, SN(k.tR, 0), SAH(k.rhs[0].Xd, i), none, 0, 1.0, 0.0},
                Prod{k.tW[1], 0, SN(k.tR, 0), SAH(k.rhs[1].Xd, i), none, 0, 1.0, 0.0}});
      // X^s_{i,i+1} = -T1 - x^s_i M^dag
      prods(s, {Prod{k.rhs[0].Xu, i, SN(k.rhs[0].Xd, i), SC(k.tM, 0), &k.tG[0], 0, -1.0, -1.0},
                Prod{k.rhs[1].Xu, i, SN(k.rhs[1].Xd, i), SC(k.tM, 0), &k.tG[1], 0, -1.0, -1.0}});
      // X^s_ii = x^s_i + T1 P^dag (+ Z - Z^dag below)
      prods(s, {Prod{k.rhs[0].Xd, i, SN(k.tG[0], 0), SC(k.tP, 0), &k.rhs[0].Xd, i, 1.0, 1.0},
                Prod{k.rhs[1].Xd, i, SN(k.tG[1], 0), SC(k.tP, 0), &k.rhs[1].Xd, i, 1.0, 1.0}});
      const View D2[2] = {k.rhs[0].Xd, k.rhs[1].Xd};
      const long long ii[2] = {i, i}, zz[2] = {0, 0};
      const View* C2[2] = {&k.rhs[0].Xd, &k.rhs[1].Xd};
      const View Z2[2] = {k.tW[0], k.tW[1]};
      s.antiherm2(2, D2, ii, C2, ii, Z2, zz, kOne, kMinus);
    } else {
      prods(s, {Prod{k.tG[0], 0, SN(k.tP, 0), SAH(k.rhs[0].Xd, i + 1), none, 0, 1.0, 0.0},
                Prod{k.tW[0], 0, SN(k.tR, 0), SAH(k.rhs[0].Xd, i), none, 0, 1.0, 0.0}});
      prods(s, {Prod{k.rhs[0].Xu, i, SN(k.rhs[0].Xd, i), SC(k.tM, 0), &k.tG[0], 0, -1.0, -1.0}});
      prods(s, {Prod{k.rhs[0].Xd, i, SN(k.tG[0], 0), SC(k.tP, 0), &k.rhs[0].Xd, i, 1.0, 1.0}});
      s.antiherm(k.rhs[0].Xd, i, &k.rhs[0].Xd, i, k.tW[0], 0, kOne, kMinus);
    }
    for (int r = 0; r < nr; ++r) {
      const Rhs& h = k.rhs[r];
      if (h.Bu.ok()) {
        // V = x_i B_{i,i+1};  X^s_{i,i+1} += V X_{i+1}^dag;  X^s_ii -= Y - Y^dag
        // with Y = V Q^dag = -V X_{i,i+1}^dag
        prods(s, {Prod{k.tY[r], 0, SN(k.xR, i), SN(h.Bu, i), none, 0, 1.0, 0.0}});
        prods(s, {Prod{h.Xu, i, SN(k.tY[r], 0), SC(k.XRd, i + 1), &h.Xu, i, 1.0, 1.0}});
        prods(s, {Prod{k.tW[r], 0, SN(k.tY[r], 0), SC(k.XRu, i), none, 0, 1.0, 0.0}});
        s.antiherm(h.Xd, i, &h.Xd, i, k.tW[r], 0, kOne, kMinus);
      }
    }
    // X^s lower = -(X^s upper)^dag
    int cnt = 0;
    View D2[2], Z2[2];
    long long ii[2] = {i, i};
    const View* C2[2] = {nullptr, nullptr};
    for (int r = 0; r < nr; ++r)
      if (k.rhs[r].Xl.ok()) { D2[cnt] = k.rhs[r].Xl; Z2[cnt] = k.rhs[r].Xu; ++cnt; }
    if (cnt) s.antiherm2(cnt, D2, ii, C2, ii, Z2, ii, kZero, kMinus);
  }
}

// ---------------------------------------------------------------- W setup --

struct WOps {
  View Vd, Vu, Vl;        // Vl empty -> use Vu with op C
  View Prd, Pru, Prl;     // per energy
  View Psd[2], Psu[2];    // per energy
  View Ad, Au, Al;        // outputs (workspace)
  View Bd[2], Bu[2];      // outputs (workspace)
  View Tm1, T0, Tp1, Tp2; // (V P^s)_{i,i-1}, _{i,i}, _{i,i+1}, _{i,i+2}
};

// Mt = I - trunc(V P^R) and B^s = trunc(V P^s V^dag); V lower = V upper^dag
// when absent, P^s lower = -(P^s upper)^dag.
void w_assemble(Emitter& s, const WOps& w, int n, int nr) {
  for (int i = 0; i < n; ++i) {
    LinCombDesc a{};
    a.idc0 = kOne;
    a.D = w.Ad.w(i); a.sD = w.Ad.es;
    s.lincomb(a);
  }
  const bool vl = w.Vl.ok();
  const char opVl = vl ? 'N' : 'C';            // V_{i+1,i} as a stored operand
  const View& VL = vl ? w.Vl : w.Vu;
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
  for (int r = 0; r < nr; ++r) {
    const View& Pd = w.Psd[r];
    const View& Pu = w.Psu[r];
    const bool pu = Pu.ok() && n > 1;
    // T0[i] = V_ii P_ii (+ V_{i,i-1} P_{i-1,i} + V_{i,i+1} P_{i+1,i})
    s.gemm('N', 'N', {Term{{w.Vd, 0}, {Pd, 0}, nullptr, 0, w.T0, 0, kOne, kZero}}, n);
    if (n > 1) {
      if (pu) {
        s.gemm(opVl, 'N', {Term{{VL, 0}, {Pu, 0}, &w.T0, 1, w.T0, 1, kOne, kOne}}, n - 1);
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

// ------------------------------------------------------------- workspace --

struct Carve {
  char* base;
  size_t off = 0;
  char* take(size_t bytes) {
    const size_t o = (off + 255) & ~size_t(255);
    off = o + bytes;
    return base ? base + o : nullptr;
  }
};

View in_view(const void* p, long long es, long long bs) {
  View v;
  v.p = (const double2*)p;
  v.es = es;
  v.bs = bs;
  return v;
}

// The lane's workspace layout; with ws == nullptr only the size is computed.
struct Layout {
  View xR, tS, tF, tP, tM, tR, tG[2], tW[2], tY[2], Uw, Lw, Hl;
  View Ad, Bd[2], Bu[2], Tm1, T0, Tp1, Tp2;
  void *panel, *brow, *spanel, *sbrow;
  int *perm, *used;
  size_t bytes;
};

Layout carve_layout(const Plan& q, int ec, char* ws) {
  Layout L{};
  Carve cv{ws};
  const int n = q.n, b = q.b;
  const long long blk = (long long)b * b;
  auto blocks = [&](long long nblk) {
    View v;
    v.p = (const double2*)cv.take((size_t)ec * nblk * blk * 16);
    v.es = nblk * blk;
    v.bs = blk;
    return v;
  };
  L.xR = blocks(n);
  L.tS = blocks(1); L.tF = blocks(1); L.tP = blocks(1); L.tM = blocks(1); L.tR = blocks(1);
  for (int r = 0; r < q.nr; ++r) {
    L.tG[r] = blocks(1);
    L.tW[r] = blocks(1);
    if (q.bt_rhs[r]) L.tY[r] = blocks(1);
  }
  if (q.general_ul && n > 1) { L.Uw = blocks(n - 1); L.Lw = blocks(n - 1); }
  if (q.need_hl) {              // H lower = H upper^dag, energy independent
    L.Hl.p = (const double2*)cv.take((size_t)(n - 1) * blk * 16);
    L.Hl.es = 0;
    L.Hl.bs = blk;
  }
  L.panel = cv.take((size_t)ec * b * kPanel * 16);
  L.brow = cv.take((size_t)ec * b * kPanel * 16);
  L.spanel = cv.take((size_t)ec * b * kSuper * 16);
  L.sbrow = cv.take((size_t)ec * b * kSuper * 16);
  L.perm = (int*)cv.take((size_t)ec * b * 4);
  L.used = (int*)cv.take((size_t)ec * b * 4);
  if (q.is_w) {
    L.Ad = blocks(n);
    for (int r = 0; r < q.nr; ++r) {
      L.Bd[r] = blocks(n);
      if (n > 1) L.Bu[r] = blocks(n - 1);
    }
    if (q.nr) { L.Tm1 = blocks(n); L.T0 = blocks(n); L.Tp1 = blocks(n); L.Tp2 = blocks(n); }
  }
  L.bytes = cv.off + 256;
  return L;
}

}  // namespace

Plan make_plan(const qtx_rgf_problem& p) {
  Plan q{};
  q.n = p.n_blocks; q.b = p.block_size; q.ne = p.n_energies;
  q.is_w = p.kind == QTX_KIND_W;
  q.fp32 = p.precision == QTX_MIXED;
  q.nr = (p.XL.diag ? 1 : 0) + (p.XG.diag ? 1 : 0);
  const int n = q.n;
  int ri = 0;
  if (!q.is_w) {
    q.general_ul = (p.S.diag && (p.S.upper || p.S.lower)) || p.sigma_r.upper || p.sigma_r.lower;
    q.need_hl = (n > 1) && !p.H.lower;
    if (p.XL.diag) q.bt_rhs[ri++] = p.sigma_l.upper != nullptr && n > 1;
    if (p.XG.diag) q.bt_rhs[ri++] = p.sigma_g.upper != nullptr && n > 1;
  } else {
    q.general_ul = true;
    for (int r = 0; r < q.nr; ++r) q.bt_rhs[r] = n > 1;
  }
  return q;
}

size_t lane_bytes(const Plan& q, int ec) { return carve_layout(q, ec, nullptr).bytes; }

void build_lane(Lane& lane, const qtx_rgf_problem& p, const Plan& q, char* ws,
                int e0, int ec, const double* d_E, int* d_info, Tuner& tuner,
                hipStream_t strm) {
  const int n = q.n, b = q.b;
  const long long blk = (long long)b * b;
  Layout lay = carve_layout(q, ec, ws);
  Emitter s(lane, tuner, strm, b, ec);
  if (q.need_hl) {
    // the lane's own copy of H lower = H upper^dagger
    Op o;
    o.k = OpK::Trans;
    o.first = (int)lane.td.size();
    for (int i = 0; i < n - 1; ++i) {
      TransDesc t{};
      t.Z = (const double2*)p.H.upper + i * blk;
      t.D = lay.Hl.w(i);
      t.a = kZero; t.z = kZero; t.g = kOne;
      t.b = b; t.batch = 1;
      lane.td.push_back(t);
    }
    o.count = (int)lane.td.size() - o.first;
    o.bytes = 32.0 * blk * (n - 1);
    lane.ops.push_back(o);
  }

  auto outv = [&](void* ptr, long long per_e) {
    View v;
    if (!ptr) return v;
    v.p = (const double2*)ptr + (long long)e0 * per_e * blk;
    v.es = per_e * blk;
    v.bs = blk;
    return v;
  };
  auto inv_ = [&](const void* ptr, long long per_e) { return outv(const_cast<void*>(ptr), per_e); };

  Core k;
  k.n = n;
  k.xR = lay.xR;
  k.tS = lay.tS; k.tF = lay.tF; k.tP = lay.tP; k.tM = lay.tM; k.tR = lay.tR;
  for (int r = 0; r < 2; ++r) { k.tG[r] = lay.tG[r]; k.tW[r] = lay.tW[r]; k.tY[r] = lay.tY[r]; }
  k.panel = lay.panel; k.brow = lay.brow; k.spanel = lay.spanel; k.sbrow = lay.sbrow;
  k.perm = lay.perm; k.used = lay.used;
  k.info = d_info + e0;
  k.XRd = outv(p.XR.diag, n);
  k.XRu = outv(p.XR.upper, n - 1);
  k.XRl = outv(p.XR.lower, n - 1);

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
      h.Bd = lay.Bd[r];
      if (n > 1) h.Bu = lay.Bu[r];
    }
    k.rhs.push_back(h);
    ++r;
  }

  if (!q.is_w) {
    const double* E = d_E + e0;
    const View Hd = in_view(p.H.diag, 0, blk);
    const View Hu = in_view(p.H.upper, 0, blk);
    const View HL = p.H.lower ? in_view(p.H.lower, 0, blk) : lay.Hl;
    const View Sd = in_view(p.S.diag, 0, blk);
    const View SRd = inv_(p.sigma_r.diag, n);
    if (q.general_ul && n > 1) {
      const View Su = in_view(p.S.upper, 0, blk), Sl = in_view(p.S.lower, 0, blk);
      const View SRu = inv_(p.sigma_r.upper, n - 1), SRl = inv_(p.sigma_r.lower, n - 1);
      for (int i = 0; i < n - 1; ++i) {
        LinCombDesc a{};
        a.E = E;
        a.src[0] = Hu.at(i); a.sSrc[0] = 0; a.c[0] = kMinus;
        if (Su.ok()) { a.src[1] = Su.at(i); a.sSrc[1] = 0; a.d[1] = kOne; }
        if (SRu.ok()) { a.src[2] = SRu.at(i); a.sSrc[2] = SRu.es; a.c[2] = kMinus; }
        a.D = lay.Uw.w(i); a.sD = lay.Uw.es;
        s.lincomb(a);
        LinCombDesc l{};
        l.E = E;
        l.src[0] = HL.at(i); l.sSrc[0] = 0; l.c[0] = kMinus;
        if (Sl.ok()) { l.src[1] = Sl.at(i); l.sSrc[1] = 0; l.d[1] = kOne; }
        if (SRl.ok()) { l.src[2] = SRl.at(i); l.sSrc[2] = SRl.es; l.c[2] = kMinus; }
        l.D = lay.Lw.w(i); l.sD = lay.Lw.es;
        s.lincomb(l);
      }
      k.U = lay.Uw; k.L = lay.Lw; k.su = 1.0; k.sl = 1.0;
    } else {
      k.U = Hu; k.L = HL; k.su = -1.0; k.sl = -1.0;
      // H Hermitian: U_i = -H_u = (-H_l)^dag and L_i = -H_l = (-H_u)^dag
      k.Uh = HL; k.suh = -1.0;
      k.Lh = Hu; k.slh = -1.0;
    }
    s.set_fp32(q.fp32);
    run_core(s, k, [&](int i) {
      LinCombDesc a{};
      a.E = E;
      if (Sd.ok()) { a.src[0] = Sd.at(i); a.sSrc[0] = 0; a.d[0] = kOne; }
      else a.idc1 = kOne;
      a.src[1] = Hd.at(i); a.sSrc[1] = 0; a.c[1] = kMinus;
      a.src[2] = SRd.at(i); a.sSrc[2] = SRd.es; a.c[2] = kMinus;
      a.D = k.tS.w(0); a.sD = k.tS.es;
      s.lincomb(a);
    });
    s.set_fp32(false);
  } else {
    WOps w{};
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
    w.Ad = lay.Ad;
    if (n > 1) { w.Au = lay.Uw; w.Al = lay.Lw; }
    for (int t = 0; t < 2; ++t) { w.Bd[t] = lay.Bd[t]; w.Bu[t] = lay.Bu[t]; }
    w.Tm1 = lay.Tm1; w.T0 = lay.T0; w.Tp1 = lay.Tp1; w.Tp2 = lay.Tp2;
    w_assemble(s, w, n, q.nr);
    k.U = w.Au; k.L = w.Al; k.su = 1.0; k.sl = 1.0;
    s.set_fp32(q.fp32);
    run_core(s, k, [&](int i) { s.copy(k.tS, 0, w.Ad, i); });
    s.set_fp32(false);
    if (p.WR_diag) {
      // W^R_ii = X_ii V_ii + X_{i,i-1} V_{i-1,i} + X_{i,i+1} V_{i+1,i}
      const View WR = outv(p.WR_diag, n);
      s.gemm('N', 'N', {Term{{k.XRd, 0}, {w.Vd, 0}, nullptr, 0, WR, 0, kOne, kZero}}, n);
      if (n > 1) {
        s.gemm('N', 'N', {Term{{k.XRl, 0}, {w.Vu, 0}, &WR, 1, WR, 1, kOne, kOne}}, n - 1);
        const bool vl = w.Vl.ok();
        s.gemm('N', vl ? 'N' : 'C', {Term{{k.XRu, 0}, {vl ? w.Vl : w.Vu, 0}, &WR, 0, WR, 0, kOne, kOne}}, n - 1);
      }
    }
  }
  lane.cls = lane_class(q, p, 2);
  lane.work = 0;
  for (const Op& o : lane.ops) lane.work += o.flops;
}

uint64_t lane_class(const Plan& q, const qtx_rgf_problem& p, int size_key) {
  // everything that shapes the operation sequence except the block count,
  // and the block size (size_key 2), a block-size bucket (1) or neither (0)
  uint64_t k = size_key == 2 ? (uint64_t)q.b : size_key == 1 ? (uint64_t)(q.b > 256) : 0;
  k = k * 2 + q.is_w;
  k = k * 2 + q.fp32;
  k = k * 2 + q.general_ul;
  k = k * 2 + q.need_hl;
  k = k * 2 + q.bt_rhs[0];
  k = k * 2 + q.bt_rhs[1];
  k = k * 4 + (uint64_t)q.nr;
  k = k * 2 + (p.WR_diag != nullptr);
  k = k * 2 + (p.S.diag != nullptr);
  k = k * 2 + (p.V.lower != nullptr);
  return k;
}

}  // namespace qtx
