// Merged-launch scheduler, descriptor arena, graph replay and autotuner.
//
// Lanes (independent solves) are advanced in rounds.  In every round the
// next operation of each unfinished lane is taken; operations with the same
// signature (kind, operand ops, precision, tile configuration) become one
// flat launch over all their descriptors, whatever the lanes' block sizes,
// block counts or positions in their recursions.  The descriptors of a
// whole segment of rounds are written into a pinned host arena, uploaded in
// one copy and launched in order on one stream, so lane order is the only
// dependency the runtime has to respect.
#include "exec.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <filesystem>
#include <fstream>
#include <functional>
#include <sstream>

namespace qtx {

#define XCHK(expr)                                  \
  do {                                              \
    hipError_t e_ = (expr);                         \
    if (e_ != hipSuccess)                           \
      throw Fail{5, std::string(#expr) + ": " +     \
                        hipGetErrorString(e_)};     \
  } while (0)

// ------------------------------------------------------------------ tuner --

std::string Tuner::cache_path() const {
  const char* p = std::getenv("QTX_TUNE_CACHE");
  if (p && *p) return p;
  const char* h = std::getenv("HOME");
  return std::string(h ? h : "/tmp") + "/.cache/qtx_rgf_tune_gfx950.json";
}

void Tuner::load() {
  loaded_ = true;
  std::ifstream f(cache_path());
  if (!f) return;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  // flat {"key": value, ...}
  size_t i = 0;
  while ((i = s.find('"', i)) != std::string::npos) {
    const size_t j = s.find('"', i + 1);
    if (j == std::string::npos) break;
    const std::string key = s.substr(i + 1, j - i - 1);
    const size_t c = s.find(':', j);
    if (c == std::string::npos) break;
    const int v = std::atoi(s.c_str() + c + 1);
    if (v >= 0 && v < kGemmConfigs) table_[key] = v;
    i = c + 1;
  }
}

void Tuner::save() const {
  const std::string p = cache_path();
  const size_t slash = p.rfind('/');
  if (slash != std::string::npos && slash > 0) {
    // in-process directory creation: no child process is started from a
    // process that has initialised the GPU
    std::error_code ec;
    std::filesystem::create_directories(p.substr(0, slash), ec);
  }
  std::ofstream f(p);
  if (!f) return;
  f << "{";
  bool first = true;
  for (auto& kv : table_) {
    f << (first ? "" : ", ") << "\"" << kv.first << "\": " << kv.second;
    first = false;
  }
  f << "}\n";
}

static int heuristic_cfg(int b) { return b <= 32 ? 2 : 0; }

int Tuner::measure(int b, bool fp32, hipStream_t s) {
  // time each configuration on a batch of b x b x b products that fills the
  // chip several times over; operands hold a nonzero byte pattern
  const long long blk = (long long)b * b;
  const int batch = std::max(1, std::min(1024, (int)(8192LL * 4096 / blk)));
  // timings are taken with the device otherwise idle (once per shape)
  XCHK(hipDeviceSynchronize());
  void* buf = nullptr;
  if (hipMalloc(&buf, (size_t)(3 * batch) * blk * 16 + 4096) != hipSuccess) {
    (void)hipGetLastError();
    return heuristic_cfg(b);
  }
  XCHK(hipMemsetAsync(buf, 0x3f, (size_t)(3 * batch) * blk * 16, s));
  GemmDesc d{};
  d.A = buf;
  d.B = (char*)buf + (size_t)batch * blk * 16;
  d.D = (char*)buf + (size_t)2 * batch * blk * 16;
  d.sA = blk; d.sB = blk; d.sD = blk;
  d.lda = b; d.ldb = b; d.ldc = b; d.ldd = b;
  d.alpha = zc{1.0, 0.0};
  d.beta = zc{0.0, 0.0};
  d.M = b; d.N = b; d.K = b;
  d.batch = batch; d.batch2 = 1;
  void* dmem = nullptr;
  XCHK(hipMalloc(&dmem, sizeof(GemmDesc) + 256));
  int* dpre = (int*)((char*)dmem + ((sizeof(GemmDesc) + 63) & ~size_t(63)));
  hipEvent_t a, z;
  XCHK(hipEventCreate(&a));
  XCHK(hipEventCreate(&z));
  float t[kGemmConfigs];
  for (int cfg = 0; cfg < kGemmConfigs; ++cfg) {
    t[cfg] = 1e30f;
    if (cfg == 1 && b < 128) continue;
    d.tiles = gemm_tiles(cfg, b, b);
    int pre[2] = {0, d.tiles * batch};
    XCHK(hipMemcpy(dmem, &d, sizeof(d), hipMemcpyHostToDevice));
    XCHK(hipMemcpy(dpre, pre, sizeof(pre), hipMemcpyHostToDevice));
    FlatLaunch l{dmem, dpre, 1, pre[1]};
    XCHK(launch_gemm(cfg, fp32, 'N', 'N', l, s));   // warm
    for (int r = 0; r < 5; ++r) {
      XCHK(hipEventRecord(a, s));
      XCHK(launch_gemm(cfg, fp32, 'N', 'N', l, s));
      XCHK(hipEventRecord(z, s));
      XCHK(hipEventSynchronize(z));
      float ms = 0;
      XCHK(hipEventElapsedTime(&ms, a, z));
      t[cfg] = std::min(t[cfg], ms);
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(z);
  (void)hipFree(dmem);
  (void)hipFree(buf);
  // the general tile unless another one is clearly faster
  int best = 0;
  for (int cfg = 1; cfg < kGemmConfigs; ++cfg)
    if (t[cfg] < 0.97f * t[best]) best = cfg;
  return best;
}

int Tuner::cfg(int M, int N, int K, bool fp32, hipStream_t s) {
  const int b = std::max(M, N);
  if (K < 32) return heuristic_cfg(std::min(b, 64));   // thin updates
  const char* force = std::getenv("QTX_GEMM_CFG");      // fixed tile for all products
  if (force && *force >= '0' && *force < '0' + kGemmConfigs) return *force - '0';
  if (!enabled_) return heuristic_cfg(b);
  std::lock_guard<std::mutex> g(mu_);
  if (!loaded_) load();
  char key[64];
  std::snprintf(key, sizeof key, "gfx950/%s/b%d", fp32 ? "c64" : "c128", b);
  auto it = table_.find(key);
  if (it != table_.end()) return it->second;
  const int c = measure(b, fp32, s);
  table_[key] = c;
  save();
  return c;
}

// ----------------------------------------------------------------- arena --

template <class D>
size_t Executor::put(const std::vector<D>& v) {
  size_t off = (host_.size() + 255) & ~size_t(255);
  host_.resize(off + v.size() * sizeof(D));
  std::memcpy(host_.data() + off, v.data(), v.size() * sizeof(D));
  return off;
}

size_t Executor::put_prefix(const std::vector<int>& p) { return put(p); }

static uint64_t fnv1a(const void* p, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* c = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ull; }
  return h;
}

// Signature: operations that may share a launch.
// Products of any shape and tile preference share a launch: every tile
// configuration accumulates each output element over k in the same order
// (chunks of four in increasing k), so the tile chosen for a launch does
// not change any result.
static uint64_t signature(const Op& o) {
  uint64_t k = (uint64_t)o.k;
  if (o.k == OpK::Gemm)
    k |= ((uint64_t)(o.opa == 'C') << 8) | ((uint64_t)(o.opb == 'C') << 9) |
         ((uint64_t)o.fp32 << 10);
  return k;
}

// Tile configuration of a merged product launch: the tuned choice of its
// largest product, moved to smaller tiles while the launch would not cover
// the chip's compute units twice.
static int group_cfg(const std::vector<std::pair<Lane*, Op*>>& ops) {
  constexpr int kFill = 2 * 256;
  const Op* big = ops[0].second;
  for (auto& lo : ops)
    if (lo.second->flops > big->flops) big = lo.second;
  auto tiles = [&](int cfg) {
    long long t = 0;
    for (auto& lo : ops)
      for (int q = 0; q < lo.second->count; ++q) {
        const GemmDesc& g = lo.first->gd[lo.second->first + q];
        t += (long long)gemm_tiles(cfg, g.M, g.N) * g.batch * std::max(1, g.batch2);
      }
    return t;
  };
  int cfg = big->cfg;
  if (cfg == 1 && tiles(1) < kFill) cfg = 0;
  if (cfg == 0 && tiles(0) < kFill) cfg = 2;
  return cfg;
}

void Executor::emit_group(std::vector<std::pair<Lane*, Op*>>& ops) {
  const Op& f = *ops[0].second;
  if (f.k == OpK::Gemm) {
    const int cfg = group_cfg(ops);
    std::vector<GemmDesc> d;
    std::vector<int> pre(1, 0);
    double fl = 0, by = 0;
    for (auto& lo : ops) {
      const Op* o = lo.second;
      for (int q = 0; q < o->count; ++q) {
        GemmDesc g = lo.first->gd[o->first + q];
        g.tiles = gemm_tiles(cfg, g.M, g.N);
        d.push_back(g);
        pre.push_back(pre.back() + g.tiles * g.batch * std::max(1, g.batch2));
      }
      fl += o->flops;
      by += o->bytes;
    }
    LaunchRec r{LaunchRec::Gemm, f.opa, f.opb, f.fp32, cfg, 0, put(d), put_prefix(pre),
                (int)d.size(), pre.back(), f.fp32 ? kClassCgemm : kClassZgemm, fl, by};
    recs_.push_back(r);
    return;
  }
  if (f.k == OpK::Inv) {
    // Matrices of b <= kSmallB: one launch of the one-workgroup inverse.
    // The others: three-level blocked Gauss-Jordan (see zinv.hip): per mega-panel, per
    // super-panel, its panels each followed by a rank-kPanel update of the
    // super-panel, then the super-panel's gather and rank-kSuper update of
    // the mega-panel's columns; after the mega-panel its gather and the
    // rank-kMega update of the columns outside it; one permutation at the end
    std::vector<InvDesc> all, small;
    double fl = 0;
    for (auto& lo : ops) {
      for (int q = 0; q < lo.second->count; ++q) {
        const InvDesc& v = lo.first->id[lo.second->first + q];
        (v.b <= kSmallB ? small : all).push_back(v);
      }
      fl += lo.second->flops;
    }
    bool first = true;
    if (!small.empty()) {
      // matrices of one workgroup's registers: the whole inverse in one launch
      std::vector<int> pre(1, 0);
      int rpl = 1;
      double by = 0;
      for (const InvDesc& v : small) {
        pre.push_back(pre.back() + v.batch);
        rpl = std::max(rpl, small_rpl(v.b));
        by += 32.0 * v.b * (double)v.b * v.batch;
      }
      recs_.push_back(LaunchRec{LaunchRec::Small, 'N', 'N', false, rpl, 0, put(small),
                                put_prefix(pre), (int)small.size(), pre.back(), kClassInv, fl, by});
      first = false;
      if (all.empty()) return;
    }
    int maxb = 0, maxn = 0;            // largest b, largest b of the one-workgroup panels
    for (auto& v : all) {
      maxb = std::max(maxb, v.b);
      if (v.b <= kTallB) maxn = std::max(maxn, v.b);
    }
    const int R = std::max(1, (maxn + kInvThreads - 1) / kInvThreads);

    auto gather_and_update = [&](int K0, int W, int cfg,
                                 const std::function<int(const InvDesc&, GemmDesc*)>& upd) {
      std::vector<InvDesc> d;
      std::vector<int> pre(1, 0);
      std::vector<GemmDesc> gd;
      std::vector<int> gpre(1, 0);
      double by = 0, gby = 0;
      for (const InvDesc& v : all) {
        GemmDesc g[2];
        const int ng = upd(v, g);
        if (ng == 0) continue;
        d.push_back(v);
        pre.push_back(pre.back() + v.batch * super_gather_chunks(v.b, W));
        by += 16.0 * 3.0 * v.b * std::min(W, v.b - K0) * v.batch;
        for (int q = 0; q < ng; ++q) {
          gd.push_back(g[q]);
          gpre.push_back(gpre.back() + g[q].tiles * g[q].batch);
          gby += 16.0 * 2.0 * g[q].M * (double)g[q].N * g[q].batch;
        }
      }
      if (d.empty()) return;
      recs_.push_back(LaunchRec{LaunchRec::Gather, 'N', 'N', false, W, K0, put(d), put_prefix(pre),
                                (int)d.size(), pre.back(), kClassInv, 0.0, by});
      recs_.push_back(LaunchRec{LaunchRec::Gemm, 'N', 'N', false, cfg, K0, put(gd),
                                put_prefix(gpre), (int)gd.size(), gpre.back(), kClassInv, 0.0, gby});
    };
    for (int M0 = 0; M0 < maxb; M0 += kMega) {
      for (int K0 = M0; K0 < std::min(M0 + kMega, maxb); K0 += kSuper) {
        for (int k0 = K0; k0 < std::min(K0 + kSuper, maxb); k0 += kPanel) {
          // one-workgroup panels (b <= kTallB) and the tournament path's
          // three steps for larger matrices, then one update launch for all
          std::vector<InvDesc> d, dt;
          std::vector<int> pre(1, 0), p1(1, 0), p2(1, 0), p3(1, 0);
          std::vector<GemmDesc> gd;
          std::vector<int> gpre(1, 0);
          double by = 0, byt = 0, gby = 0;
          for (const InvDesc& v : all) {
            if (v.b <= k0) continue;
            if (v.b <= kTallB) {
              d.push_back(v);
              pre.push_back(pre.back() + v.batch);
              by += 16.0 * 3.0 * v.b * kPanel * v.batch;
            } else {
              dt.push_back(v);
              p1.push_back(p1.back() + v.batch * tall_chunks(v.b));
              p2.push_back(p2.back() + v.batch);
              p3.push_back(p3.back() + v.batch * ((v.b + kInvThreads - 1) / kInvThreads));
              byt += 16.0 * 4.0 * v.b * kPanel * v.batch;
            }
            GemmDesc g;
            if (inv_panel_update(v, k0, &g)) {
              gd.push_back(g);
              gpre.push_back(gpre.back() + g.tiles * g.batch);
              gby += 16.0 * 2.0 * g.M * (double)g.N * g.batch;
            }
          }
          if (!d.empty()) {
            recs_.push_back(LaunchRec{LaunchRec::Panel, 'N', 'N', false, R, k0, put(d),
                                      put_prefix(pre), (int)d.size(), pre.back(), kClassInv,
                                      (first ? fl : 0.0), by});
            first = false;
          }
          if (!dt.empty()) {
            const size_t off = put(dt);
            const LaunchRec::Kind kinds[3] = {LaunchRec::TallSelect, LaunchRec::TallFinal,
                                              LaunchRec::TallApply};
            const std::vector<int>* pres[3] = {&p1, &p2, &p3};
            for (int st = 0; st < 3; ++st) {
              recs_.push_back(LaunchRec{kinds[st], 'N', 'N', false, 0, k0, off, put_prefix(*pres[st]),
                                        (int)dt.size(), pres[st]->back(), kClassInv,
                                        (first ? fl : 0.0), st == 0 ? byt : 0.0});
              first = false;
            }
          }
          if (!gd.empty())
            recs_.push_back(LaunchRec{LaunchRec::Gemm, 'N', 'N', false, kGemmInvUpdate, k0, put(gd),
                                      put_prefix(gpre), (int)gd.size(), gpre.back(), kClassInv, 0.0,
                                      gby});
        }
        // rank-kSuper update of the mega-panel's other columns
        gather_and_update(K0, kSuper, kGemmInvUpdate, [&](const InvDesc& v, GemmDesc* g) {
          return inv_super_update(v, K0, g) ? 1 : 0;
        });
      }
      // rank-kMega update of the columns outside the mega-panel
      gather_and_update(M0, kMega, kMegaCfg, [&](const InvDesc& v, GemmDesc* g) {
        int ng = 0;
        for (int side = 0; side < 2; ++side)
          if (inv_mega_update(v, M0, side, &g[ng])) ++ng;
        return ng;
      });
    }
    std::vector<int> pre(1, 0);
    double by = 0;
    for (const InvDesc& v : all) {
      pre.push_back(pre.back() + v.batch * ((v.b + kPermRows - 1) / kPermRows));
      by += 32.0 * v.b * (double)v.b * v.batch;
    }
    recs_.push_back(LaunchRec{LaunchRec::Permute, 'N', 'N', false, 0, 0, put(all), put_prefix(pre),
                              (int)all.size(), pre.back(), kClassInv, 0.0, by});
    return;
  }
  if (f.k == OpK::Lin) {
    std::vector<LinCombDesc> d;
    std::vector<int> pre(1, 0);
    double by = 0;
    for (auto& lo : ops) {
      for (int q = 0; q < lo.second->count; ++q) {
        const LinCombDesc& v = lo.first->ld[lo.second->first + q];
        d.push_back(v);
        pre.push_back(pre.back() + v.batch * lincomb_chunks(v.b));
      }
      by += lo.second->bytes;
    }
    recs_.push_back(LaunchRec{LaunchRec::Lin, 'N', 'N', false, 0, 0, put(d), put_prefix(pre),
                              (int)d.size(), pre.back(), kClassElem, 0.0, by});
    return;
  }
  std::vector<TransDesc> d;
  std::vector<int> pre(1, 0);
  double by = 0;
  for (auto& lo : ops) {
    for (int q = 0; q < lo.second->count; ++q) {
      const TransDesc& v = lo.first->td[lo.second->first + q];
      d.push_back(v);
      pre.push_back(pre.back() + v.batch * trans_tiles(v.b));
    }
    by += lo.second->bytes;
  }
  recs_.push_back(LaunchRec{LaunchRec::Trans, 'N', 'N', false, 0, 0, put(d), put_prefix(pre),
                            (int)d.size(), pre.back(), kClassElem, 0.0, by});
}

int Executor::build(std::vector<Lane*>& lanes, size_t arena_limit, int max_rounds,
                    bool stop_on_finish, int max_launches) {
  int rounds = 0;
  struct Head { uint64_t sig; Lane* l; Op* o; };
  std::vector<Head> heads;
  std::vector<std::pair<Lane*, Op*>> grp;
  while (host_.size() < arena_limit && rounds < max_rounds) {
    heads.clear();
    for (Lane* l : lanes)
      if (!l->done()) heads.push_back(Head{signature(l->ops[l->next]), l, &l->ops[l->next]});
    if (heads.empty()) break;
    std::stable_sort(heads.begin(), heads.end(),
                     [](const Head& a, const Head& b) { return a.sig < b.sig; });
    size_t i = 0;
    while (i < heads.size()) {
      size_t j = i;
      grp.clear();
      while (j < heads.size() && heads[j].sig == heads[i].sig) {
        grp.push_back({heads[j].l, heads[j].o});
        ++j;
      }
      emit_group(grp);
      i = j;
    }
    bool fin = false;
    for (Lane* l : lanes)
      if (!l->done()) {
        l->next++;
        fin |= l->done();
      }
    ++rounds;
    if (fin && stop_on_finish) break;
    if ((int)recs_.size() >= max_launches) break;
  }
  return rounds;
}

hipEvent_t Executor::get_event() {
  if (!ev_pool_.empty()) {
    hipEvent_t e = ev_pool_.back();
    ev_pool_.pop_back();
    return e;
  }
  hipEvent_t e;
  XCHK(hipEventCreate(&e));
  return e;
}

void Executor::issue(char* base, bool profile) {
  for (const LaunchRec& r : recs_) {
    FlatLaunch l{base + r.desc_off, (const int*)(base + r.prefix_off), r.nd, r.total};
    hipEvent_t a = nullptr, b = nullptr;
    if (profile) {
      a = get_event();
      b = get_event();
      XCHK(hipEventRecord(a, s_));
    }
    switch (r.kind) {
      case LaunchRec::Gemm: XCHK(launch_gemm(r.cfg, r.fp32, r.opa, r.opb, l, s_)); break;
      case LaunchRec::Panel: XCHK(launch_inv_panel(r.cfg, r.k0, l, s_)); break;
      case LaunchRec::TallSelect: XCHK(launch_inv_tall(1, r.k0, l, s_)); break;
      case LaunchRec::TallFinal: XCHK(launch_inv_tall(2, r.k0, l, s_)); break;
      case LaunchRec::TallApply: XCHK(launch_inv_tall(3, r.k0, l, s_)); break;
      case LaunchRec::Permute: XCHK(launch_inv_permute(l, s_)); break;
      case LaunchRec::Small: XCHK(launch_inv_small(r.cfg, l, s_)); break;
      case LaunchRec::Gather: XCHK(launch_inv_super_gather(r.k0, r.cfg, l, s_)); break;
      case LaunchRec::Lin: XCHK(launch_lincomb(l, s_)); break;
      case LaunchRec::Trans: XCHK(launch_transcomb(l, s_)); break;
    }
    if (profile) {
      XCHK(hipEventRecord(b, s_));
      pending_.push_back(Pending{r.cls, a, b, r.flops, r.bytes});
    }
  }
}

void Executor::flush(bool profile, bool graphs, std::vector<KStat>& stats) {
  if (recs_.empty()) {
    host_.clear();
    return;
  }
  const size_t bytes = host_.size();
  uint64_t key = 0;
  if (graphs && !profile) {
    key = fnv1a(host_.data(), bytes);
    key = fnv1a(recs_.data(), recs_.size() * sizeof(LaunchRec), key);
    auto it = graphs_.find(key);
    if (it != graphs_.end()) {
      it->second.last = ++tick_;
      XCHK(hipGraphLaunch(it->second.exec, s_));
      recs_.clear();
      host_.clear();
      return;
    }
    if (++seen_[key] >= 2 && graphs_.size() < 64) {
      // second sight of this segment: capture it with its own arena
      GraphEntry g{};
      XCHK(hipMalloc((void**)&g.arena, bytes));
      XCHK(hipMemcpyAsync(g.arena, host_.data(), bytes, hipMemcpyHostToDevice, s_));
      XCHK(hipStreamSynchronize(s_));
      hipGraph_t graph;
      XCHK(hipStreamBeginCapture(s_, hipStreamCaptureModeThreadLocal));
      issue(g.arena, false);
      XCHK(hipStreamEndCapture(s_, &graph));
      XCHK(hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0));
      (void)hipGraphDestroy(graph);
      g.bytes = bytes;
      g.last = ++tick_;
      graphs_[key] = g;
      XCHK(hipGraphLaunch(g.exec, s_));
      recs_.clear();
      host_.clear();
      return;
    }
  }
  // eager: pinned staging + device arena, double-buffered by slot
  const int sl = slot_;
  slot_ ^= 1;
  if (done_[sl]) XCHK(hipEventSynchronize(done_[sl]));
  if (pin_cap_[sl] < bytes) {
    if (pin_[sl]) (void)hipHostFree(pin_[sl]);
    pin_cap_[sl] = std::max(bytes, (size_t)1 << 20);
    XCHK(hipHostMalloc((void**)&pin_[sl], pin_cap_[sl], 0));
  }
  if (dev_cap_[sl] < bytes) {
    if (dev_[sl]) {
      XCHK(hipStreamSynchronize(s_));
      (void)hipFree(dev_[sl]);
    }
    dev_cap_[sl] = std::max(bytes, (size_t)1 << 20);
    XCHK(hipMalloc((void**)&dev_[sl], dev_cap_[sl]));
  }
  std::memcpy(pin_[sl], host_.data(), bytes);
  XCHK(hipMemcpyAsync(dev_[sl], pin_[sl], bytes, hipMemcpyHostToDevice, s_));
  issue(dev_[sl], profile);
  if (!done_[sl]) XCHK(hipEventCreateWithFlags(&done_[sl], hipEventDisableTiming));
  XCHK(hipEventRecord(done_[sl], s_));
  recs_.clear();
  host_.clear();
  if (pending_.size() > 8192) sync_and_collect(stats);
}

void Executor::sync_and_collect(std::vector<KStat>& stats) {
  XCHK(hipStreamSynchronize(s_));
  for (auto& p : pending_) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      KStat& s = stats[p.cls];
      s.launches += 1;
      s.ms += ms;
      s.flops += p.flops;
      s.bytes += p.bytes;
    }
    ev_pool_.push_back(p.a);
    ev_pool_.push_back(p.b);
  }
  pending_.clear();
}

void Executor::release() {
  (void)hipStreamSynchronize(s_);
  for (auto& kv : graphs_) {
    (void)hipGraphExecDestroy(kv.second.exec);
    (void)hipFree(kv.second.arena);
  }
  graphs_.clear();
  seen_.clear();
  for (int i = 0; i < 2; ++i) {
    if (dev_[i]) (void)hipFree(dev_[i]);
    if (pin_[i]) (void)hipHostFree(pin_[i]);
    if (done_[i]) (void)hipEventDestroy(done_[i]);
    dev_[i] = nullptr; pin_[i] = nullptr; done_[i] = nullptr;
    dev_cap_[i] = pin_cap_[i] = 0;
  }
  for (auto& p : pending_) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
  pending_.clear();
  for (auto e : ev_pool_) (void)hipEventDestroy(e);
  ev_pool_.clear();
}

Executor::~Executor() { release(); }

bool Executor::slot_ready() const {
  const hipEvent_t e = done_[slot_];
  return !e || hipEventQuery(e) == hipSuccess;
}

void Executor::wait_slot() {
  if (done_[slot_]) XCHK(hipEventSynchronize(done_[slot_]));
}

// ------------------------------------------------------------------- pool --

Pool::Pool(hipStream_t main, int n) {
  n = std::max(1, n);
  x_.resize(n);
  try {
    for (int i = 0; i < n; ++i) {
      X& x = x_[i];
      if (i == 0) {
        x.s = main;
      } else {
        XCHK(hipStreamCreateWithFlags(&x.s, hipStreamNonBlocking));
        x.own = true;
      }
      x.exe.reset(new Executor(x.s));
      XCHK(hipEventCreateWithFlags(&x.rel, hipEventDisableTiming));
      XCHK(hipEventCreateWithFlags(&x.ev, hipEventDisableTiming));
      x.waited.assign(n, 0);
    }
  } catch (...) {
    destroy();                     // the destructor does not run for a failed constructor
    throw;
  }
}

void Pool::destroy() {
  for (X& x : x_) {
    if (x.s) (void)hipStreamSynchronize(x.s);
    x.exe.reset();
    if (x.rel) (void)hipEventDestroy(x.rel);
    if (x.ev) (void)hipEventDestroy(x.ev);
    if (x.own && x.s) (void)hipStreamDestroy(x.s);
    x = X();
  }
}

Pool::~Pool() { destroy(); }

int Pool::place(uint64_t cls) {
  auto it = cls_x_.find(cls);
  if (it != cls_x_.end()) return it->second;
  int best = 0;
  for (int i = 1; i < size(); ++i)
    if (x_[i].load < x_[best].load) best = i;
  return best;
}

void Pool::add(Lane* l, int xi) {
  X& x = x_[xi];
  for (int j = 0; j < size(); ++j) {
    if (j == xi || x_[j].rel_count == x.waited[j]) continue;
    XCHK(hipStreamWaitEvent(x.s, x_[j].rel, 0));
    x.waited[j] = x_[j].rel_count;
  }
  x.lanes.push_back(l);
  x.load += l->work;
  cls_x_[l->cls] = xi;
  cls_n_[l->cls]++;
}

bool Pool::busy() const {
  for (const X& x : x_)
    if (!x.lanes.empty()) return true;
  return false;
}

void Pool::step(size_t arena_limit, int max_rounds, bool stop_on_finish, bool profile,
                bool graphs, std::vector<KStat>& stats,
                std::vector<std::pair<Lane*, int>>& done) {
  bool issued = false;
  int first_busy = -1, n_busy = 0;
  for (const X& x : x_) n_busy += !x.lanes.empty();
  const int cap = n_busy > 1 ? kPoolSegLaunches : (1 << 30);
  for (int i = 0; i < size(); ++i) {
    X& x = x_[i];
    if (x.lanes.empty()) continue;
    if (!x.exe->slot_ready()) {
      if (first_busy < 0) first_busy = i;
      continue;
    }
    x.exe->build(x.lanes, arena_limit, max_rounds, stop_on_finish, cap);
    x.exe->flush(profile, graphs, stats);
    issued = true;
    bool fin = false;
    for (size_t k = 0; k < x.lanes.size();) {
      Lane* l = x.lanes[k];
      if (l->done()) {
        done.push_back({l, i});
        x.load -= l->work;
        if (--cls_n_[l->cls] == 0) {
          cls_n_.erase(l->cls);
          cls_x_.erase(l->cls);
        }
        x.lanes.erase(x.lanes.begin() + k);
        fin = true;
      } else {
        ++k;
      }
    }
    if (x.lanes.empty()) x.load = 0;
    if (fin) {
      XCHK(hipEventRecord(x.rel, x.s));
      x.rel_count++;
    }
  }
  if (!issued && first_busy >= 0) x_[first_busy].exe->wait_slot();
}

void Pool::fork() {
  if (size() == 1) return;
  XCHK(hipEventRecord(x_[0].ev, x_[0].s));
  for (int i = 1; i < size(); ++i) XCHK(hipStreamWaitEvent(x_[i].s, x_[0].ev, 0));
}

void Pool::join() {
  for (int i = 1; i < size(); ++i) {
    XCHK(hipEventRecord(x_[i].ev, x_[i].s));
    XCHK(hipStreamWaitEvent(x_[0].s, x_[i].ev, 0));
  }
}

void Pool::sync_and_collect(std::vector<KStat>& stats) {
  for (X& x : x_) x.exe->sync_and_collect(stats);
}

void Pool::sync() {
  for (X& x : x_) XCHK(hipStreamSynchronize(x.s));
}

void Pool::release() {
  for (X& x : x_) x.exe->release();
}

}  // namespace qtx
