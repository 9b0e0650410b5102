// The partitioned solve of Sec. 4.4 (Fig. nested-dissection) on one device:
// per-partition elimination with fill-in, the reduced system on the
// separators, per-partition recovery of the selected blocks.
//
// Partition p holds blocks [lo, hi).  Its elimination chain lists its
// interior blocks in elimination order and ends at the separator N that the
// chain runs into:
//   top     chain lo .. hi-2 (top-down),   N = hi-1;
//   bottom  chain hi-1 .. lo+1 (bottom-up), N = lo;
//   middle  chain lo+1 .. hi-2 (top-down), N = hi-1, and the anchor T = lo,
//           the partition's other separator, which stays while the chain is
//           eliminated.
// In chain order the couplings are Uc(k) = Mt_{c_k, c_{k+1}} and
// Lc(k) = Mt_{c_{k+1}, c_k} (for the bottom chain the upper and lower blocks
// of Mt trade places).  Eliminating c_k (x_k = inverse of its current
// diagonal block) updates the next block as in the plain forward pass and,
// in a middle partition, the fill-in that couples the chain to T:
//   q_{k+1} = Mt_{c_{k+1},T} = -Lc(k) x_k q_k,   q_0 = Mt_{c_0,T},
//   r_{k+1} = Mt_{T,c_{k+1}} = -r_k x_k Uc(k),   r_0 = Mt_{T,c_0},
//   Mt_TT  -= r_k x_k q_k,
// and for each right-hand side (anti-Hermitian, carried as L^{-1} B L^{-dag})
//   rho_{k+1} = R_{c_{k+1},T} = -Lc(k) x_k rho_k + Bc(k)^dag (r_k x_k)^dag
//               + Lc(k) x^s_k r_k^dag,           rho_0 = B_{c_0,T},
//   R_TT += -Z + Z^dag + r_k x^s_k r_k^dag,        Z = r_k x_k rho_k.
// The last step writes the separators' blocks of the reduced system (and
// the fill-in coupling T-N).  The backward step of a chain block recovers
// it from the blocks of its neighbours N_k = {c_{k+1}, T}:
//   X_{k,N} = -x_k Mt_{k,N} X_NN,  X_{N,k} = -X_NN Mt_{N,k} x_k,
//   X_kk = x_k + x_k Mt_{k,N} X_NN Mt_{N,k} x_k,
//   X^s_{k,N} = -x_k Mt_{k,N} X^s_NN - x^s_k (X_NN Mt_{N,k})^dag + x_k R_{k,N} X_NN^dag,
//   X^s_kk = x^s_k + P X^s_NN P^dag + (Z - Z^dag) + (Y - Y^dag),
//   P = x_k Mt_{k,N},  Z = P X_NN Mt_{N,k} x^s_k,  Y = x_k R_{k,N} X_{k,N}^dag,
// the relations of Sec. 3.2.3 with the single neighbour replaced by the
// pair {c_{k+1}, T}; without an anchor they are the plain backward pass.
#include <algorithm>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "../../include/qtx_rgf.h"
#include "ctx.h"
#include "emit.h"
#include "emitter.h"

namespace qtx {
namespace {

// Contiguous partition sizes: n / P, the first n % P one larger.
bool partition_ranges(int n, int P, std::vector<int>& lo, std::vector<int>& hi) {
  if (P < 2) return false;
  lo.assign(P, 0);
  hi.assign(P, 0);
  int at = 0;
  for (int p = 0; p < P; ++p) {
    const int sz = n / P + (p < n % P ? 1 : 0);
    const bool ok = (p == 0 || p == P - 1) ? sz >= 1 : sz >= 2;
    if (!ok) return false;
    lo[p] = at;
    hi[p] = at + sz;
    at += sz;
  }
  return true;
}

struct Chain {
  std::vector<int> c;   // interior blocks in elimination order
  int N = 0;            // the separator the chain runs into
  int T = -1;           // anchor separator (middle partitions), -1 none
  bool rev = false;     // bottom partition: the chain runs upwards
  int jN = 0, jT = -1;  // separator indices in the reduced system
  int m() const { return (int)c.size(); }
  int g(int k) const { return k < m() ? c[k] : N; }
};

Chain make_chain(int p, int P, int lo, int hi) {
  Chain ch;
  if (p == 0) {
    for (int i = lo; i < hi - 1; ++i) ch.c.push_back(i);
    ch.N = hi - 1;
    ch.jN = 0;
  } else if (p == P - 1) {
    for (int i = hi - 1; i > lo; --i) ch.c.push_back(i);
    ch.N = lo;
    ch.rev = true;
    ch.jN = 2 * P - 3;
  } else {
    for (int i = lo + 1; i < hi - 1; ++i) ch.c.push_back(i);
    ch.N = hi - 1;
    ch.T = lo;
    ch.jT = 2 * p - 1;
    ch.jN = 2 * p;
  }
  return ch;
}

// Temporaries and inverse buffers of one partition (one block per energy each).
struct Temps {
  View tS, tF, tRT, tP, tPT, tM, tMT, tR;
  View tG[2], tG2[2], tW[2], tW2[2], tY[2], tQ[2], tRho[2], tZ[2], tXs[2];
  void *panel, *brow, *spanel, *sbrow;
  int *perm, *used;
};

struct NLayout {
  // indexed by global block
  View xR, Qf, Rf, XkT, XTk, RHO[2], XSkT[2];
  // reduced system: separators' blocks, right-hand sides, solution
  View Sd, Su, Sl, Rd[2], Ru[2], Yd, Yu, Yl, YSd[2], YSu[2], xRr;
  // assembled operands, as in the plain lane
  View Uw, Lw, Hl, Ad, Bd[2], Bu[2], Tm1, T0, Tp1, Tp2;
  std::vector<Temps> pt;
  size_t bytes = 0;
};

NLayout carve_nested(const Plan& q, int P, int ec, char* ws) {
  NLayout L;
  Carve cv{ws};
  const int n = q.n, b = q.b, ns = 2 * P - 2;
  const long long blk = (long long)b * b;
  auto blocks = [&](long long nblk) {
    View v;
    v.p = (const double2*)cv.take((size_t)ec * nblk * blk * 16);
    v.es = nblk * blk;
    v.bs = blk;
    return v;
  };
  L.xR = blocks(n);
  L.Qf = blocks(n); L.Rf = blocks(n); L.XkT = blocks(n); L.XTk = blocks(n);
  for (int r = 0; r < q.nr; ++r) { L.RHO[r] = blocks(n); L.XSkT[r] = blocks(n); }
  L.Sd = blocks(ns); L.Su = blocks(ns - 1); L.Sl = blocks(ns - 1);
  for (int r = 0; r < q.nr; ++r) { L.Rd[r] = blocks(ns); L.Ru[r] = blocks(ns - 1); }
  L.Yd = blocks(ns); L.Yu = blocks(ns - 1); L.Yl = blocks(ns - 1);
  for (int r = 0; r < q.nr; ++r) { L.YSd[r] = blocks(ns); L.YSu[r] = blocks(ns - 1); }
  L.xRr = blocks(ns);
  if (q.general_ul) { L.Uw = blocks(n - 1); L.Lw = blocks(n - 1); }
  if (q.need_hl) {
    L.Hl.p = (const double2*)cv.take((size_t)(n - 1) * blk * 16);
    L.Hl.es = 0;
    L.Hl.bs = blk;
  }
  if (q.is_w) {
    L.Ad = blocks(n);
    for (int r = 0; r < q.nr; ++r) { L.Bd[r] = blocks(n); L.Bu[r] = blocks(n - 1); }
    if (q.nr) { L.Tm1 = blocks(n); L.T0 = blocks(n); L.Tp1 = blocks(n); L.Tp2 = blocks(n); }
  }
  L.pt.resize(P);
  for (int p = 0; p < P; ++p) {
    Temps& t = L.pt[p];
    t.tS = blocks(1); t.tF = blocks(1); t.tRT = blocks(1); t.tP = blocks(1);
    t.tPT = blocks(1); t.tM = blocks(1); t.tMT = blocks(1); t.tR = blocks(1);
    for (int r = 0; r < q.nr; ++r) {
      t.tG[r] = blocks(1); t.tG2[r] = blocks(1); t.tW[r] = blocks(1); t.tW2[r] = blocks(1);
      t.tY[r] = blocks(1); t.tQ[r] = blocks(1); t.tRho[r] = blocks(1); t.tZ[r] = blocks(1);
      t.tXs[r] = blocks(1);
    }
    t.panel = cv.take((size_t)ec * b * kPanel * 16);
    t.brow = cv.take((size_t)ec * b * kPanel * 16);
    t.spanel = cv.take((size_t)ec * b * inv_span(b) * 16);
    t.sbrow = cv.take((size_t)ec * b * inv_span(b) * 16);
    t.perm = (int*)cv.take((size_t)ec * b * 4);
    t.used = (int*)cv.take((size_t)ec * b * 4);
  }
  L.bytes = cv.off + 256;
  return L;
}

// The assembled system as operand accessors: couplings of Mt (read through
// an adjoint relation where one exists, as in the plain lane), the diagonal
// blocks written on demand, the right-hand sides and the outputs.
struct Sys {
  View U, L, Uh, Lh;
  double su = 1.0, sl = 1.0, suh = 1.0, slh = 1.0;
  int nr = 0;
  View Bd[2], Bu[2];          // Bu empty: block-diagonal right-hand side
  View XRd, XRu, XRl;
  View Xd[2], Xu[2], Xl[2];   // Xl may be empty
  std::function<void(Emitter&, const View&, long long, int)> prep;   // D[id] = Mt_ii
  Src Ur(long long i) const { return Uh.ok() ? SC(Uh, i, suh) : SN(U, i, su); }
  Src Lr(long long i) const { return Lh.ok() ? SC(Lh, i, slh) : SN(L, i, sl); }
};

const View* const none = nullptr;

void prod(Emitter& s, const View& D, long long id, const Src& a, const Src& b, const View* C,
          long long ic, double alpha, double beta) {
  prods(s, {Prod{D, id, a, b, C, ic, alpha, beta}});
}

// D[id] = value of the operand a
void put_src(Emitter& s, const View& D, long long id, const Src& a) {
  if (a.op == 'N') {
    LinCombDesc l{};
    l.src[0] = a.v.at(a.i); l.sSrc[0] = a.v.es; l.c[0] = rs(a.sg);
    l.D = D.w(id); l.sD = D.es;
    s.lincomb(l);
  } else {
    s.antiherm(D, id, nullptr, 0, a.v, a.i, kZero, rs(a.sg));
  }
}
void put_zero(Emitter& s, const View& D, long long id) {
  LinCombDesc l{};
  l.D = D.w(id); l.sD = D.es;
  s.lincomb(l);
}
// D[id] = -(Z[iz])^dagger
void put_neg_adj(Emitter& s, const View& D, long long id, const View& Z, long long iz) {
  s.antiherm(D, id, nullptr, 0, Z, iz, kZero, kMinus);
}

struct Ctx {
  Emitter& s;
  const Sys& y;
  const NLayout& L;
  const Temps& t;
  const Chain& ch;
  int* info;
  Src Uc(int k) const { const int g = ch.g(k); return ch.rev ? y.Lr(g - 1) : y.Ur(g); }
  Src Lc(int k) const { const int g = ch.g(k); return ch.rev ? y.Ur(g - 1) : y.Lr(g); }
  bool Bc(int r, int k, Src* out) const {
    if (!y.Bu[r].ok()) return false;
    const int g = ch.g(k);
    *out = ch.rev ? Src{y.Bu[r], g - 1, 'C', -1.0} : SN(y.Bu[r], g);
    return true;
  }
  Src qsrc(int k) const { return k == 0 ? y.Lr(ch.T) : SN(L.Qf, ch.g(k)); }
  Src rsrc(int k) const { return k == 0 ? y.Ur(ch.T) : SN(L.Rf, ch.g(k)); }
  bool rhosrc(int r, int k, Src* out) const {
    if (k > 0) { *out = SN(L.RHO[r], ch.g(k)); return true; }
    if (!y.Bu[r].ok()) return false;
    *out = Src{y.Bu[r], ch.T, 'C', -1.0};        // B_{T+1,T} = -B_{T,T+1}^dag
    return true;
  }
  void inv(int g) {
    s.inverse(t.tS, 0, L.xR, g, t.panel, t.brow, t.spanel, t.sbrow, t.perm, t.used, info,
              g + 1, false);
  }
};

// ---- phase 1: forward elimination of one partition -----------------------
void emit_forward(Ctx& x) {
  Emitter& s = x.s;
  const Sys& y = x.y;
  const NLayout& L = x.L;
  const Temps& t = x.t;
  const Chain& ch = x.ch;
  const int m = ch.m(), T = ch.T;
  const bool anc = T >= 0;
  if (m == 0) {
    y.prep(s, L.Sd, ch.jN, ch.N);
    for (int r = 0; r < y.nr; ++r) s.copy(L.Rd[r], ch.jN, y.Bd[r], ch.N);
    if (anc) {                     // two adjacent separators, no interior
      y.prep(s, L.Sd, ch.jT, T);
      put_src(s, L.Su, ch.jT, y.Ur(T));
      put_src(s, L.Sl, ch.jT, y.Lr(T));
      for (int r = 0; r < y.nr; ++r) {
        s.copy(L.Rd[r], ch.jT, y.Bd[r], T);
        if (y.Bu[r].ok()) s.copy(L.Ru[r], ch.jT, y.Bu[r], T);
        else put_zero(s, L.Ru[r], ch.jT);
      }
    }
    return;
  }
  const int c0 = ch.c[0];
  y.prep(s, t.tS, 0, c0);
  x.inv(c0);
  for (int r = 0; r < y.nr; ++r) {
    prod(s, t.tG[r], 0, SN(L.xR, c0), SAH(y.Bd[r], c0), none, 0, 1.0, 0.0);
    prod(s, y.Xd[r], c0, SN(t.tG[r], 0), SC(L.xR, c0), none, 0, 1.0, 0.0);
  }
  if (anc) {
    y.prep(s, L.Sd, ch.jT, T);
    for (int r = 0; r < y.nr; ++r) s.copy(L.Rd[r], ch.jT, y.Bd[r], T);
  }
  for (int k = 0; k < m; ++k) {
    const int c = ch.g(k), nx = ch.g(k + 1);
    const bool last = k + 1 == m;
    // F = Lc x_k;  next diagonal block minus F Uc
    prod(s, t.tF, 0, x.Lc(k), SN(L.xR, c), none, 0, 1.0, 0.0);
    if (!last) {
      y.prep(s, t.tS, 0, nx);
      prod(s, t.tS, 0, SN(t.tF, 0), x.Uc(k), &t.tS, 0, -1.0, 1.0);
      x.inv(nx);
    } else {
      y.prep(s, L.Sd, ch.jN, ch.N);
      prod(s, L.Sd, ch.jN, SN(t.tF, 0), x.Uc(k), &L.Sd, ch.jN, -1.0, 1.0);
    }
    if (anc) {
      // fill-in: l_T = r_k x_k, q_{k+1}, r_{k+1}, Mt_TT
      prod(s, t.tRT, 0, x.rsrc(k), SN(L.xR, c), none, 0, 1.0, 0.0);
      const View& qd = last ? L.Sl : L.Qf;
      const View& rd = last ? L.Su : L.Rf;
      const long long qi = last ? ch.jT : nx;
      prods(s, {Prod{qd, qi, SN(t.tF, 0), x.qsrc(k), none, 0, -1.0, 0.0},
                Prod{rd, qi, SN(t.tRT, 0), x.Uc(k), none, 0, -1.0, 0.0}});
      prod(s, L.Sd, ch.jT, SN(t.tRT, 0), x.qsrc(k), &L.Sd, ch.jT, -1.0, 1.0);
    }
    for (int r = 0; r < y.nr; ++r) {
      // W = B_nx + Lc x^s_k Lc^dag - y + y^dag,  y = F Bc
      prod(s, t.tG[r], 0, x.Lc(k), SAH(y.Xd[r], c), none, 0, 1.0, 0.0);
      if (anc) prod(s, t.tRho[r], 0, SN(t.tG[r], 0), adj(x.rsrc(k)), none, 0, 1.0, 0.0);
      const View& Wv = last ? L.Rd[r] : t.tW[r];
      const long long wi = last ? ch.jN : 0;
      prod(s, Wv, wi, SN(t.tG[r], 0), adj(x.Lc(k)), &y.Bd[r], nx, 1.0, 1.0);
      Src bc;
      const bool hb = x.Bc(r, k, &bc);
      if (hb) {
        prod(s, t.tY[r], 0, SN(t.tF, 0), bc, none, 0, 1.0, 0.0);
        s.antiherm(Wv, wi, &Wv, wi, t.tY[r], 0, kMinus, kOne);
      }
      if (!last) {
        prod(s, t.tG[r], 0, SN(L.xR, nx), SAH(t.tW[r], 0), none, 0, 1.0, 0.0);
        prod(s, y.Xd[r], nx, SN(t.tG[r], 0), SC(L.xR, nx), none, 0, 1.0, 0.0);
      }
      if (anc) {
        const View& rhod = last ? t.tQ[r] : L.RHO[r];
        const long long rhoi = last ? 0 : nx;
        Src rho;
        const bool hr = x.rhosrc(r, k, &rho);
        if (hr) prod(s, rhod, rhoi, SN(t.tF, 0), rho, &t.tRho[r], 0, -1.0, 1.0);
        else s.copy(rhod, rhoi, t.tRho[r], 0);
        if (hb) prod(s, rhod, rhoi, adj(bc), SC(t.tRT, 0), &rhod, rhoi, 1.0, 1.0);
        if (hr) {
          prod(s, t.tZ[r], 0, SN(t.tRT, 0), rho, none, 0, 1.0, 0.0);
          s.antiherm(L.Rd[r], ch.jT, &L.Rd[r], ch.jT, t.tZ[r], 0, kMinus, kOne);
        }
        prod(s, t.tG2[r], 0, x.rsrc(k), SAH(y.Xd[r], c), none, 0, 1.0, 0.0);
        prod(s, L.Rd[r], ch.jT, SN(t.tG2[r], 0), adj(x.rsrc(k)), &L.Rd[r], ch.jT, 1.0, 1.0);
        if (last) put_neg_adj(s, L.Ru[r], ch.jT, rhod, rhoi);
      }
    }
  }
}

// ---- phase 3: backward recovery of one partition --------------------------
void emit_backward(Ctx& x, int P, int p, int hi_p) {
  Emitter& s = x.s;
  const Sys& y = x.y;
  const NLayout& L = x.L;
  const Temps& t = x.t;
  const Chain& ch = x.ch;
  const int m = ch.m(), T = ch.T;
  const bool anc = T >= 0;
  // the separators' own blocks, and the coupling to the next partition
  s.copy(y.XRd, ch.N, L.Yd, ch.jN);
  for (int r = 0; r < y.nr; ++r) s.copy(y.Xd[r], ch.N, L.YSd[r], ch.jN);
  if (anc) {
    s.copy(y.XRd, T, L.Yd, ch.jT);
    for (int r = 0; r < y.nr; ++r) s.copy(y.Xd[r], T, L.YSd[r], ch.jT);
  }
  if (p < P - 1) {
    const int i = hi_p - 1, j = 2 * p;
    s.copy(y.XRu, i, L.Yu, j);
    s.copy(y.XRl, i, L.Yl, j);
    for (int r = 0; r < y.nr; ++r) {
      s.copy(y.Xu[r], i, L.YSu[r], j);
      if (y.Xl[r].ok()) put_neg_adj(s, y.Xl[r], i, L.YSu[r], j);
    }
  }
  if (m == 0) {
    if (anc) {                     // T and N adjacent
      s.copy(y.XRu, T, L.Yu, ch.jT);
      s.copy(y.XRl, T, L.Yl, ch.jT);
      for (int r = 0; r < y.nr; ++r) {
        s.copy(y.Xu[r], T, L.YSu[r], ch.jT);
        if (y.Xl[r].ok()) put_neg_adj(s, y.Xl[r], T, L.YSu[r], ch.jT);
      }
    }
    return;
  }
  for (int k = m - 1; k >= 0; --k) {
    const int c = ch.g(k), nx = ch.g(k + 1);
    const bool last = k + 1 == m;
    // the pair (c, nx) in the outputs: upper/lower of the lower block index
    const View& Xcn = ch.rev ? y.XRl : y.XRu;
    const View& Xnc = ch.rev ? y.XRu : y.XRl;
    const long long pi = ch.rev ? nx : c;
    if (!anc) {
      prods(s, {Prod{t.tP, 0, SN(L.xR, c), x.Uc(k), none, 0, 1.0, 0.0},
                Prod{t.tM, 0, SN(y.XRd, nx), x.Lc(k), none, 0, 1.0, 0.0}});
      prods(s, {Prod{Xcn, pi, SN(t.tP, 0), SN(y.XRd, nx), none, 0, -1.0, 0.0},
                Prod{Xnc, pi, SN(t.tM, 0), SN(L.xR, c), none, 0, -1.0, 0.0}});
      prod(s, t.tR, 0, SN(Xcn, pi), x.Lc(k), none, 0, -1.0, 0.0);
    } else {
      const Src XrT = last ? SN(L.Yl, ch.jT) : SN(L.XkT, nx);
      const Src XTr = last ? SN(L.Yu, ch.jT) : SN(L.XTk, nx);
      const Src XTT = SN(y.XRd, T);
      prods(s, {Prod{t.tP, 0, SN(L.xR, c), x.Uc(k), none, 0, 1.0, 0.0},
                Prod{t.tPT, 0, SN(L.xR, c), x.qsrc(k), none, 0, 1.0, 0.0},
                Prod{t.tM, 0, SN(y.XRd, nx), x.Lc(k), none, 0, 1.0, 0.0},
                Prod{t.tMT, 0, XTr, x.Lc(k), none, 0, 1.0, 0.0}});
      prods(s, {Prod{Xcn, pi, SN(t.tP, 0), SN(y.XRd, nx), none, 0, -1.0, 0.0},
                Prod{L.XkT, c, SN(t.tP, 0), XrT, none, 0, -1.0, 0.0},
                Prod{t.tM, 0, XrT, x.rsrc(k), &t.tM, 0, 1.0, 1.0},
                Prod{t.tMT, 0, XTT, x.rsrc(k), &t.tMT, 0, 1.0, 1.0}});
      prods(s, {Prod{Xcn, pi, SN(t.tPT, 0), XTr, &Xcn, pi, -1.0, 1.0},
                Prod{L.XkT, c, SN(t.tPT, 0), XTT, &L.XkT, c, -1.0, 1.0},
                Prod{Xnc, pi, SN(t.tM, 0), SN(L.xR, c), none, 0, -1.0, 0.0},
                Prod{L.XTk, c, SN(t.tMT, 0), SN(L.xR, c), none, 0, -1.0, 0.0}});
      prod(s, t.tR, 0, SN(Xcn, pi), x.Lc(k), none, 0, -1.0, 0.0);
      prod(s, t.tR, 0, SN(L.XkT, c), x.rsrc(k), &t.tR, 0, -1.0, 1.0);
    }
    // lesser/greater first: they read the forward x^s_k and x_k; then X_kk
    for (int r = 0; r < y.nr; ++r) {
      const View& Xs = ch.rev ? t.tXs[r] : y.Xu[r];     // X^s_{c,nx}
      const long long xi = ch.rev ? 0 : c;
      Src bc;
      const bool hb = x.Bc(r, k, &bc);
      if (!anc) {
        prods(s, {Prod{t.tG[r], 0, SN(t.tP, 0), SAH(y.Xd[r], nx), none, 0, 1.0, 0.0},
                  Prod{t.tW[r], 0, SN(t.tR, 0), SAH(y.Xd[r], c), none, 0, 1.0, 0.0}});
        prod(s, Xs, xi, SN(y.Xd[r], c), SC(t.tM, 0), &t.tG[r], 0, -1.0, -1.0);
        if (hb) {
          prod(s, t.tY[r], 0, SN(L.xR, c), bc, none, 0, 1.0, 0.0);
          prods(s, {Prod{Xs, xi, SN(t.tY[r], 0), SC(y.XRd, nx), &Xs, xi, 1.0, 1.0},
                    Prod{t.tW2[r], 0, SN(t.tY[r], 0), SC(Xcn, pi), none, 0, 1.0, 0.0}});
        }
        prod(s, y.Xd[r], c, SN(t.tG[r], 0), SC(t.tP, 0), &y.Xd[r], c, 1.0, 1.0);
        s.antiherm(y.Xd[r], c, &y.Xd[r], c, t.tW[r], 0, kOne, kMinus);
        if (hb) s.antiherm(y.Xd[r], c, &y.Xd[r], c, t.tW2[r], 0, kOne, kMinus);
      } else {
        const Src XrT = last ? SN(L.Yl, ch.jT) : SN(L.XkT, nx);
        const Src XTr = last ? SN(L.Yu, ch.jT) : SN(L.XTk, nx);
        const Src XTT = SN(y.XRd, T);
        const Src XsrT = last ? Src{L.YSu[r], ch.jT, 'C', -1.0} : SN(L.XSkT[r], nx);
        const Src XsTr = last ? SN(L.YSu[r], ch.jT) : Src{L.XSkT[r], nx, 'C', -1.0};
        const Src XsTT = SN(y.Xd[r], T);
        Src rho;
        const bool hr = x.rhosrc(r, k, &rho);
        prods(s, {Prod{t.tW[r], 0, SN(t.tR, 0), SAH(y.Xd[r], c), none, 0, 1.0, 0.0},
                  Prod{t.tG[r], 0, SN(t.tP, 0), SAH(y.Xd[r], nx), none, 0, 1.0, 0.0},
                  Prod{t.tG2[r], 0, SN(t.tP, 0), XsrT, none, 0, 1.0, 0.0}});
        prods(s, {Prod{t.tG[r], 0, SN(t.tPT, 0), XsTr, &t.tG[r], 0, 1.0, 1.0},
                  Prod{t.tG2[r], 0, SN(t.tPT, 0), XsTT, &t.tG2[r], 0, 1.0, 1.0}});
        prods(s, {Prod{Xs, xi, SN(y.Xd[r], c), SC(t.tM, 0), &t.tG[r], 0, -1.0, -1.0},
                  Prod{L.XSkT[r], c, SN(y.Xd[r], c), SC(t.tMT, 0), &t.tG2[r], 0, -1.0, -1.0}});
        bool w2 = false;
        if (hb) {
          prod(s, t.tY[r], 0, SN(L.xR, c), bc, none, 0, 1.0, 0.0);
          prods(s, {Prod{Xs, xi, SN(t.tY[r], 0), SC(y.XRd, nx), &Xs, xi, 1.0, 1.0},
                    Prod{L.XSkT[r], c, SN(t.tY[r], 0), adj(XTr), &L.XSkT[r], c, 1.0, 1.0},
                    Prod{t.tW2[r], 0, SN(t.tY[r], 0), SC(Xcn, pi), none, 0, 1.0, 0.0}});
          w2 = true;
        }
        if (hr) {
          prod(s, t.tQ[r], 0, SN(L.xR, c), rho, none, 0, 1.0, 0.0);
          prods(s, {Prod{Xs, xi, SN(t.tQ[r], 0), adj(XrT), &Xs, xi, 1.0, 1.0},
                    Prod{L.XSkT[r], c, SN(t.tQ[r], 0), adj(XTT), &L.XSkT[r], c, 1.0, 1.0},
                    Prod{t.tW2[r], 0, SN(t.tQ[r], 0), SC(L.XkT, c), w2 ? &t.tW2[r] : none, 0,
                         1.0, w2 ? 1.0 : 0.0}});
          w2 = true;
        }
        prod(s, y.Xd[r], c, SN(t.tG[r], 0), SC(t.tP, 0), &y.Xd[r], c, 1.0, 1.0);
        prod(s, y.Xd[r], c, SN(t.tG2[r], 0), SC(t.tPT, 0), &y.Xd[r], c, 1.0, 1.0);
        s.antiherm(y.Xd[r], c, &y.Xd[r], c, t.tW[r], 0, kOne, kMinus);
        if (w2) s.antiherm(y.Xd[r], c, &y.Xd[r], c, t.tW2[r], 0, kOne, kMinus);
      }
      // the other triangle of the pair
      if (!ch.rev) {
        if (y.Xl[r].ok()) put_neg_adj(s, y.Xl[r], c, y.Xu[r], c);
      } else {
        put_neg_adj(s, y.Xu[r], nx, t.tXs[r], 0);
        if (y.Xl[r].ok()) s.copy(y.Xl[r], nx, t.tXs[r], 0);
      }
    }
    prod(s, y.XRd, c, SN(t.tR, 0), SN(L.xR, c), &L.xR, c, 1.0, 1.0);
    if (anc && k == 0) {           // the pair (T, c_0): upper / lower block T
      s.copy(y.XRu, T, L.XTk, c);
      s.copy(y.XRl, T, L.XkT, c);
      for (int r = 0; r < y.nr; ++r) {
        if (y.Xl[r].ok()) s.copy(y.Xl[r], T, L.XSkT[r], c);
        put_neg_adj(s, y.Xu[r], T, L.XSkT[r], c);
      }
    }
  }
}

}  // namespace
}  // namespace qtx

using namespace qtx;

namespace {

size_t nested_bytes(const Plan& q, int P, int ec) { return carve_nested(q, P, ec, nullptr).bytes; }

// One energy chunk: lanes of the four phases, each phase run to completion.
void nested_chunk(qtx_rgf_ctx* c, const qtx_rgf_problem& p, const qtx_rgf_nested& o,
                  const Plan& q, int e0, int ec, const double* d_E, int* d_info) {
  const int n = q.n, b = q.b, P = o.n_partitions, ns = 2 * P - 2;
  const long long blk = (long long)b * b;
  NLayout L = carve_nested(q, P, ec, c->ws);
  std::vector<int> lo, hi;
  partition_ranges(n, P, lo, hi);
  hipStream_t st = c->pool->stream(0);

  auto outv = [&](const void* ptr, long long per_e) {
    View v;
    if (!ptr) return v;
    v.p = (const double2*)ptr + (long long)e0 * per_e * blk;
    v.es = per_e * blk;
    v.bs = blk;
    return v;
  };
  Sys y;
  y.XRd = outv(p.XR.diag, n);
  y.XRu = outv(p.XR.upper, n - 1);
  y.XRl = outv(p.XR.lower, n - 1);
  const qtx_bt_out* outs[2] = {&p.XL, &p.XG};
  int rr = 0;
  for (int tt = 0; tt < 2; ++tt) {
    if (!outs[tt]->diag) continue;
    y.Xd[rr] = outv(outs[tt]->diag, n);
    y.Xu[rr] = outv(outs[tt]->upper, n - 1);
    y.Xl[rr] = outv(outs[tt]->lower, n - 1);
    ++rr;
  }
  y.nr = q.nr;

  // ---- phase 0: assembled operands -------------------------------------
  std::vector<std::unique_ptr<Lane>> lanes;
  auto new_lane = [&]() {
    lanes.emplace_back(new Lane());
    lanes.back()->e0 = e0;
    lanes.back()->ec = ec;
    return lanes.back().get();
  };
  auto run = [&](std::vector<Lane*> ls) { run_lanes_to_end(c, ls); };
  {
    Lane* l0 = new_lane();
    Emitter s(*l0, c->tuner, st, b, ec);
    if (q.need_hl) {
      // H lower = H upper^dagger, energy independent: one matrix per block
      Op op;
      op.k = OpK::Trans;
      op.first = (int)l0->td.size();
      for (int i = 0; i < n - 1; ++i) {
        TransDesc t{};
        t.Z = (const double2*)p.H.upper + i * blk;
        t.D = L.Hl.w(i);
        t.a = kZero; t.z = kZero; t.g = kOne;
        t.b = b; t.batch = 1;
        l0->td.push_back(t);
      }
      op.count = (int)l0->td.size() - op.first;
      op.bytes = 32.0 * blk * (n - 1);
      l0->ops.push_back(op);
    }
    if (!q.is_w) {
      const double* E = d_E + e0;
      const View Hd = in_view(p.H.diag, 0, blk);
      const View Hu = in_view(p.H.upper, 0, blk);
      const View HL = p.H.lower ? in_view(p.H.lower, 0, blk) : L.Hl;
      const View Sd = in_view(p.S.diag, 0, blk);
      const View SRd = outv(p.sigma_r.diag, n);
      if (q.general_ul) {
        const View Su = in_view(p.S.upper, 0, blk), Sl = in_view(p.S.lower, 0, blk);
        const View SRu = outv(p.sigma_r.upper, n - 1), SRl = outv(p.sigma_r.lower, n - 1);
        for (int i = 0; i < n - 1; ++i) {
          LinCombDesc a{};
          a.E = E;
          a.src[0] = Hu.at(i); a.sSrc[0] = 0; a.c[0] = kMinus;
          if (Su.ok()) { a.src[1] = Su.at(i); a.sSrc[1] = 0; a.d[1] = kOne; }
          if (SRu.ok()) { a.src[2] = SRu.at(i); a.sSrc[2] = SRu.es; a.c[2] = kMinus; }
          a.D = L.Uw.w(i); a.sD = L.Uw.es;
          s.lincomb(a);
          LinCombDesc l{};
          l.E = E;
          l.src[0] = HL.at(i); l.sSrc[0] = 0; l.c[0] = kMinus;
          if (Sl.ok()) { l.src[1] = Sl.at(i); l.sSrc[1] = 0; l.d[1] = kOne; }
          if (SRl.ok()) { l.src[2] = SRl.at(i); l.sSrc[2] = SRl.es; l.c[2] = kMinus; }
          l.D = L.Lw.w(i); l.sD = L.Lw.es;
          s.lincomb(l);
        }
        y.U = L.Uw; y.L = L.Lw;
      } else {
        // H Hermitian: U_i = -H_u = (-H_l)^dag and L_i = -H_l = (-H_u)^dag
        y.U = Hu; y.L = HL; y.su = -1.0; y.sl = -1.0;
        y.Uh = HL; y.suh = -1.0;
        y.Lh = Hu; y.slh = -1.0;
      }
      y.prep = [E, Sd, Hd, SRd](Emitter& em, const View& D, long long id, int i) {
        LinCombDesc a{};
        a.E = E;
        if (Sd.ok()) { a.src[0] = Sd.at(i); a.sSrc[0] = 0; a.d[0] = kOne; }
        else a.idc1 = kOne;
        a.src[1] = Hd.at(i); a.sSrc[1] = 0; a.c[1] = kMinus;
        a.src[2] = SRd.at(i); a.sSrc[2] = SRd.es; a.c[2] = kMinus;
        a.D = D.w(id); a.sD = D.es;
        em.lincomb(a);
      };
      const qtx_bt_in* Bs[2] = {&p.sigma_l, &p.sigma_g};
      int r = 0;
      for (int tt = 0; tt < 2; ++tt) {
        if (!outs[tt]->diag) continue;
        y.Bd[r] = outv(Bs[tt]->diag, n);
        if (Bs[tt]->upper && n > 1) y.Bu[r] = outv(Bs[tt]->upper, n - 1);
        ++r;
      }
    } else {
      WOps w{};
      w.Vd = in_view(p.V.diag, 0, blk);
      w.Vu = in_view(p.V.upper, 0, blk);
      w.Vl = in_view(p.V.lower, 0, blk);
      w.Prd = outv(p.P_r.diag, n);
      w.Pru = outv(p.P_r.upper, n - 1);
      w.Prl = outv(p.P_r.lower, n - 1);
      const qtx_bt_in* Ps[2] = {&p.P_l, &p.P_g};
      int r = 0;
      for (int tt = 0; tt < 2; ++tt) {
        if (!outs[tt]->diag) continue;
        w.Psd[r] = outv(Ps[tt]->diag, n);
        w.Psu[r] = outv(Ps[tt]->upper, n - 1);
        ++r;
      }
      w.Ad = L.Ad;
      w.Au = L.Uw; w.Al = L.Lw;
      for (int tt = 0; tt < 2; ++tt) { w.Bd[tt] = L.Bd[tt]; w.Bu[tt] = L.Bu[tt]; }
      w.Tm1 = L.Tm1; w.T0 = L.T0; w.Tp1 = L.Tp1; w.Tp2 = L.Tp2;
      w_assemble(s, w, n, q.nr);
      y.U = L.Uw; y.L = L.Lw;
      const View Ad = L.Ad;
      y.prep = [Ad](Emitter& em, const View& D, long long id, int i) { em.copy(D, id, Ad, i); };
      for (int t2 = 0; t2 < q.nr; ++t2) { y.Bd[t2] = L.Bd[t2]; y.Bu[t2] = L.Bu[t2]; }
    }
    if (!l0->ops.empty()) run({l0});
  }

  std::vector<Chain> chains(P);
  for (int pp = 0; pp < P; ++pp) chains[pp] = make_chain(pp, P, lo[pp], hi[pp]);
  int* info = d_info + e0;

  // ---- phase 1: every partition's forward elimination --------------------
  {
    std::vector<Lane*> ls;
    for (int pp = 0; pp < P; ++pp) {
      Lane* l = new_lane();
      Emitter s(*l, c->tuner, st, b, ec);
      s.set_fp32(q.fp32);
      Ctx x{s, y, L, L.pt[pp], chains[pp], info};
      emit_forward(x);
      s.set_fp32(false);
      if (pp < P - 1) {            // original coupling to the next partition
        const int i = hi[pp] - 1, j = 2 * pp;
        put_src(s, L.Su, j, y.Ur(i));
        put_src(s, L.Sl, j, y.Lr(i));
        for (int r = 0; r < q.nr; ++r) {
          if (y.Bu[r].ok()) s.copy(L.Ru[r], j, y.Bu[r], i);
          else put_zero(s, L.Ru[r], j);
        }
      }
      ls.push_back(l);
    }
    run(ls);
  }

  // ---- phase 2: the reduced system --------------------------------------
  {
    Lane* l = new_lane();
    Emitter s(*l, c->tuner, st, b, ec);
    const qtx_bt_out* red[3] = {&o.reduced, &o.reduced_l, &o.reduced_g};
    if (red[0]->diag) {
      for (int j = 0; j < ns; ++j) s.copy(outv(red[0]->diag, ns), j, L.Sd, j);
      for (int j = 0; j < ns - 1; ++j) {
        if (red[0]->upper) s.copy(outv(red[0]->upper, ns - 1), j, L.Su, j);
        if (red[0]->lower) s.copy(outv(red[0]->lower, ns - 1), j, L.Sl, j);
      }
    }
    int r = 0;
    for (int tt = 0; tt < 2; ++tt) {
      if (!outs[tt]->diag) continue;
      const qtx_bt_out* ro = red[1 + tt];
      if (ro->diag) {
        for (int j = 0; j < ns; ++j) s.copy(outv(ro->diag, ns), j, L.Rd[r], j);
        if (ro->upper)
          for (int j = 0; j < ns - 1; ++j) s.copy(outv(ro->upper, ns - 1), j, L.Ru[r], j);
      }
      ++r;
    }
    std::vector<int> seps;
    for (int pp = 0; pp < P; ++pp) {
      if (pp > 0) seps.push_back(chains[pp].T >= 0 ? chains[pp].T : chains[pp].N);
      if (pp < P - 1) seps.push_back(chains[pp].N);
    }
    std::vector<int> codes(ns);
    for (int j = 0; j < ns; ++j) codes[j] = seps[j] + 1;
    Core k;
    k.n = ns;
    k.U = L.Su; k.L = L.Sl;
    k.xR = L.xRr;
    const Temps& t = L.pt[0];
    k.tS = t.tS; k.tF = t.tF; k.tP = t.tP; k.tM = t.tM; k.tR = t.tR;
    for (int r2 = 0; r2 < q.nr; ++r2) { k.tG[r2] = t.tG[r2]; k.tW[r2] = t.tW[r2]; k.tY[r2] = t.tY[r2]; }
    k.panel = t.panel; k.brow = t.brow; k.spanel = t.spanel; k.sbrow = t.sbrow;
    k.perm = t.perm; k.used = t.used;
    k.info = info;
    k.code = codes.data();
    k.reset_info = false;
    k.XRd = L.Yd; k.XRu = L.Yu; k.XRl = L.Yl;
    for (int r2 = 0; r2 < q.nr; ++r2) {
      Rhs h;
      h.Bd = L.Rd[r2]; h.Bu = L.Ru[r2];
      h.Xd = L.YSd[r2]; h.Xu = L.YSu[r2];
      k.rhs.push_back(h);
    }
    s.set_fp32(q.fp32);
    run_core(s, k, [&](int i) {
      LinCombDesc a{};          // the reduced system's diagonal block
      a.src[0] = L.Sd.at(i); a.sSrc[0] = L.Sd.es; a.c[0] = kOne;
      return a;
    });
    s.set_fp32(false);
    run({l});
  }

  // ---- phase 3: every partition's backward recovery ----------------------
  {
    std::vector<Lane*> ls;
    for (int pp = 0; pp < P; ++pp) {
      Lane* l = new_lane();
      Emitter s(*l, c->tuner, st, b, ec);
      s.set_fp32(q.fp32);
      Ctx x{s, y, L, L.pt[pp], chains[pp], info};
      emit_backward(x, P, pp, hi[pp]);
      s.set_fp32(false);
      ls.push_back(l);
    }
    run(ls);
  }
  if (q.is_w && p.WR_diag) {
    // W^R_ii = X_ii V_ii + X_{i,i-1} V_{i-1,i} + X_{i,i+1} V_{i+1,i}
    Lane* l = new_lane();
    Emitter s(*l, c->tuner, st, b, ec);
    const View WR = outv(p.WR_diag, n);
    const View Vd = in_view(p.V.diag, 0, blk), Vu = in_view(p.V.upper, 0, blk);
    const View Vl = in_view(p.V.lower, 0, blk);
    s.gemm('N', 'N', {Term{{y.XRd, 0}, {Vd, 0}, nullptr, 0, WR, 0, kOne, kZero}}, n);
    if (n > 1) {
      s.gemm('N', 'N', {Term{{y.XRl, 0}, {Vu, 0}, &WR, 1, WR, 1, kOne, kOne}}, n - 1);
      const bool vl = Vl.ok();
      s.gemm('N', vl ? 'N' : 'C', {Term{{y.XRu, 0}, {vl ? Vl : Vu, 0}, &WR, 0, WR, 0, kOne, kOne}}, n - 1);
    }
    run({l});
  }
}

qtx_status solve_nested(qtx_rgf_ctx* c, qtx_rgf_problem& p, const qtx_rgf_nested& o) {
  p.status = QTX_OK;
  p.fail_energy = -1;
  p.fail_block = -1;
  const Plan q = make_plan(p);
  const int ne = q.ne;
  const size_t eb = (((size_t)ne * 8) + 255) & ~size_t(255);
  const size_t ib = (((size_t)ne * 4) + 255) & ~size_t(255);
  ensure(c, &c->aux, &c->aux_bytes, eb + ib + 256);
  double* d_E = (double*)c->aux;
  int* d_info = (int*)(c->aux + eb);
  hipStream_t st = c->pool->stream(0);
  {
    std::vector<double> hE(ne, 0.0);
    if (p.kind == QTX_KIND_G) std::memcpy(hE.data(), p.energies, sizeof(double) * ne);
    HIPCHK(c, hipMemcpyAsync(d_E, hE.data(), sizeof(double) * ne, hipMemcpyHostToDevice, st));
    // the partitions' inverses of one energy share launches: the status
    // words are cleared once here and only failures are written
    HIPCHK(c, hipMemsetAsync(d_info, 0, sizeof(int) * ne, st));
    HIPCHK(c, hipStreamSynchronize(st));
  }
  const size_t budget = budget_now(c);
  const int P = o.n_partitions;
  if (nested_bytes(q, P, 1) > budget) {
    c->err = "one energy needs " + std::to_string(nested_bytes(q, P, 1)) +
             " workspace bytes, budget is " + std::to_string(budget);
    throw Fail{QTX_ERR_NOMEM};
  }
  int lo = 1, hi = ne;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (nested_bytes(q, P, mid) <= budget) lo = mid; else hi = mid - 1;
  }
  ensure(c, &c->ws, &c->ws_bytes, nested_bytes(q, P, lo) + 4096);
  for (int e0 = 0; e0 < ne; e0 += lo)
    nested_chunk(c, p, o, q, e0, std::min(lo, ne - e0), d_E, d_info);
  std::vector<int> h_info(ne);
  HIPCHK(c, hipMemcpyAsync(h_info.data(), d_info, sizeof(int) * ne, hipMemcpyDeviceToHost, st));
  c->pool->exe(0).sync_and_collect(c->stats);
  HIPCHK(c, hipStreamSynchronize(st));
  for (int e = 0; e < ne; ++e) {
    const int v = h_info[e];
    if (v != 0) {
      p.status = v > 0 ? QTX_ERR_SINGULAR : QTX_ERR_NOT_FINITE;
      p.fail_energy = e;
      p.fail_block = std::abs(v) - 1;
      return QTX_ERR_PROBLEM;
    }
  }
  return QTX_OK;
}

}  // namespace

extern "C" qtx_status qtx_rgf_solve_nested(qtx_rgf_ctx* c, qtx_rgf_problem* p,
                                           const qtx_rgf_nested* o) {
  if (!c) return QTX_ERR_INVALID_ARG;
  if (c->busy) return QTX_ERR_BUSY;
  c->err.clear();
  if (!p || !o) { c->err = "problem and options are required"; return QTX_ERR_INVALID_ARG; }
  const std::string m = validate_problem(*p);
  if (!m.empty()) { c->err = m; return QTX_ERR_INVALID_ARG; }
  std::vector<int> lo, hi;
  if (!partition_ranges(p->n_blocks, o->n_partitions, lo, hi)) {
    c->err = "cannot split " + std::to_string(p->n_blocks) + " blocks into " +
             std::to_string(o->n_partitions) +
             " partitions (>= 2 partitions; middle ones need >= 2 blocks)";
    return QTX_ERR_INVALID_ARG;
  }
  const qtx_bt_out* red[3] = {&o->reduced, &o->reduced_l, &o->reduced_g};
  for (int i = 0; i < 3; ++i)
    if (red[i]->diag && (!red[i]->upper || (i == 0 && !red[i]->lower))) {
      c->err = "a reduced-system output needs its upper (and, for the matrix, lower) blocks";
      return QTX_ERR_INVALID_ARG;
    }
  if ((o->reduced_l.diag && !p->XL.diag) || (o->reduced_g.diag && !p->XG.diag)) {
    c->err = "reduced right-hand side requested for an output that is not computed";
    return QTX_ERR_INVALID_ARG;
  }
  c->busy = true;
  qtx_status st;
  try {
    HIPCHK(c, hipSetDevice(c->device));
    st = solve_nested(c, *p, *o);
  } catch (const Fail& f) {
    if (c->err.empty()) c->err = f.what;
    try { c->pool->sync_and_collect(c->stats); } catch (...) {}
    st = (qtx_status)f.st;
  } catch (...) {
    c->err = "internal error";
    st = QTX_ERR_HIP;
  }
  c->busy = false;
  return st;
}
