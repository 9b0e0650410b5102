// Building blocks of the lane emitters (emit.cpp: the RGF recursion of one
// lane; nested.cpp: the partitioned scheme): block-indexed operand views,
// the emitter that turns block products, inverses and elementwise passes
// into lane operations, and the forward/backward recursion on a block
// chain (arXiv 2508.19138, Sec. 3.2.3, Eqs. forward-pass / backward-pass).
//
// Notation: x_i = x^R_i (left-connected), xs_i = x^s_i, X_i = X^R_i,
// U_i = Mt_{i,i+1}, L_i = Mt_{i+1,i}.  The right-hand sides are
// anti-Hermitian, so each of  y - y^dag,  Y - Y^dag  and  Z - Z^dag  needs a
// single product, and the lower blocks of X^s are -upper^dagger.
#pragma once
#include <initializer_list>

#include "exec.h"

namespace qtx {

inline const zc kOne{1.0, 0.0}, kZero{0.0, 0.0}, kMinus{-1.0, 0.0};
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

  // D = alpha * op(A) op(B) + C with C assembled in the product's epilogue
  // from the linear combination `c` (its D and batch fields are unused).
  void gemm_asm(char opa, char opb, const Opnd& A, const Opnd& B, const View& D, long long id,
                zc alpha, const LinCombDesc& c) {
    Op o;
    o.k = OpK::Gemm;
    o.opa = opa; o.opb = opb; o.fp32 = fp32_;
    o.cfg = T_.cfg(b_, b_, b_, fp32_, s_);
    o.first = (int)L_.gd.size();
    GemmDesc g{};
    g.A = A.v.at(A.i); g.sA = A.v.es; g.tA = A.v.bs;
    g.B = B.v.at(B.i); g.sB = B.v.es; g.tB = B.v.bs;
    g.D = D.w(id); g.sD = D.es; g.tD = D.bs;
    g.lda = g.ldb = g.ldc = g.ldd = b_;
    g.alpha = alpha;
    g.beta = kZero;
    g.M = g.N = g.K = b_;
    g.batch = ec_;
    g.batch2 = 1;
    g.asm_ = 1;
    for (int t = 0; t < 3; ++t) {
      g.X[t] = c.src[t]; g.sX[t] = c.sSrc[t];
      g.xc[t] = c.c[t]; g.xd[t] = c.d[t];
    }
    g.i0 = c.idc0; g.i1 = c.idc1;
    g.E = c.E;
    L_.gd.push_back(g);
    o.count = 1;
    o.flops = 8.0 * blk_ * b_ * (double)ec_;
    int nsrc = 0;
    for (int t = 0; t < 3; ++t) nsrc += c.src[t] != nullptr;
    o.bytes = 16.0 * blk_ * (3.0 + nsrc) * ec_;
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
  // status code of a failing inverse of block i: code[i] if given, else i + 1
  const int* code = nullptr;
  bool reset_info = true;    // the first inverse clears the status words
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
// the adjoint of an operand
inline Src adj(const Src& a) { return Src{a.v, a.i, a.op == 'N' ? 'C' : 'N', a.sg}; }

struct Prod {             // D = alpha * a b + beta * C
  View D;
  long long id;
  Src a, b;
  const View* C;
  long long ic;
  double alpha, beta;
};

// Emit independent products; those sharing operand ops share one operation.
inline void prods(Emitter& s, std::initializer_list<Prod> ps) {
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

// Forward and backward passes, given a callback that describes Mt_ii as a
// linear combination (LinCombDesc without destination).  Mt_00 is written by
// an elementwise pass; every later Mt_ii is assembled in the epilogue of the
// Schur update Mt_ii - F U_{i-1} (no separate pass, no extra block in HBM).
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
              k.code ? k.code[i] : i + 1, i == 0 && k.reset_info);
  };
  const View* none = nullptr;

  // ---- forward pass ----------------------------------------------------
  {
    LinCombDesc a = prep_diag(0);
    a.D = k.tS.w(0); a.sD = k.tS.es;
    s.lincomb(a);
  }
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
    {
      const Src u = Ur(i - 1);
      s.gemm_asm('N', u.op, Opnd{k.tF, 0}, Opnd{u.v, u.i}, k.tS, 0, rs(-u.sg), prep_diag(i));
    }
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

// Mt = I - trunc(V P^R) and B^s = trunc(V P^s V^dag) (emit.cpp).
void w_assemble(Emitter& s, const WOps& w, int n, int nr);

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

inline View in_view(const void* p, long long es, long long bs) {
  View v;
  v.p = (const double2*)p;
  v.es = es;
  v.bs = bs;
  return v;
}

}  // namespace qtx
