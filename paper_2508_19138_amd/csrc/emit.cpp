// The RGF recursion of one lane as a list of block operations
// (arXiv 2508.19138, Sec. 3.2.3, Eqs. forward-pass / backward-pass; system
// assembly of Sec. 3.2.2 and Table "quantities"); the recursion itself is
// run_core in emitter.h.
#include "emit.h"

#include <algorithm>

#include "emitter.h"

namespace qtx {

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

namespace {

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
  L.spanel = cv.take((size_t)ec * b * inv_span(b) * 16);
  L.sbrow = cv.take((size_t)ec * b * inv_span(b) * 16);
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
      LinCombDesc a{};          // Mt_ii = E S_ii - H_ii - Sigma^R_ii
      a.E = E;
      if (Sd.ok()) { a.src[0] = Sd.at(i); a.sSrc[0] = 0; a.d[0] = kOne; }
      else a.idc1 = kOne;
      a.src[1] = Hd.at(i); a.sSrc[1] = 0; a.c[1] = kMinus;
      a.src[2] = SRd.at(i); a.sSrc[2] = SRd.es; a.c[2] = kMinus;
      return a;
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
    run_core(s, k, [&](int i) {
      LinCombDesc a{};          // Mt_ii as assembled by w_assemble
      a.src[0] = w.Ad.at(i); a.sSrc[0] = w.Ad.es; a.c[0] = kOne;
      return a;
    });
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
