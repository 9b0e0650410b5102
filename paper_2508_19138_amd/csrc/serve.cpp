// Request loop of the RGF library: continuous batching of independently
// submitted problems (qtx_rgf_submit / qtx_rgf_poll).
//
// A host thread owns its own HIP streams, workspace and launch arenas.  It
// admits queued problems in arrival order, energy chunk by chunk, whenever
// workspace frees up, and advances every admitted lane in merged launches
// (exec.cpp): lanes of one shape class share launches on one stream and
// different classes run concurrently on the others, so problems that arrive
// while others run join the next segment of launches and overlap with them.
// A segment is cut as soon as a lane finishes so that its workspace can be
// handed to the next problem.  A problem completes when the events recorded
// after each of its lanes' last operations have completed.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <thread>
#include <unordered_map>

#include "ctx.h"
#include "emit.h"

namespace qtx {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t ticket = 0;
  qtx_rgf_problem p{};
  std::vector<double> E;
  Plan q;
  Clock::time_point t_sub, t_adm;
  bool admitted_any = false;
  size_t aux_off = 0, aux_len = 0;
  bool has_aux = false;
  double* dE = nullptr;
  int* dinfo = nullptr;
  int next_e0 = 0;
  int ec_max = 1;
  int lanes_out = 0;        // lanes issued whose work is not yet complete
};

class Server {
 public:
  Server(qtx_rgf_ctx* c, size_t ws_budget);
  ~Server();
  qtx_status submit(const qtx_rgf_problem& p, uint64_t* ticket);
  qtx_status poll(qtx_rgf_completion* out, int cap, int* n, int* pending, int wait_ms);

 private:
  struct Fin {
    hipEvent_t ev;          // recorded after the lane's last operation
    Request* r;
  };
  void loop();
  void admit();
  void retire(bool block);
  void complete(Request* r);
  void fail_all(int st);
  void free_resources();
  hipEvent_t get_event();

  qtx_rgf_ctx* c_;
  std::thread th_;
  std::mutex mu_;
  std::condition_variable cv_in_, cv_out_;
  std::deque<std::unique_ptr<Request>> incoming_;
  std::deque<qtx_rgf_completion> done_;
  bool stop_ = false;
  bool failed_ = false;
  uint64_t next_ticket_ = 1;
  int outstanding_ = 0;

  // owned by the loop thread
  hipStream_t s_ = nullptr, s_read_ = nullptr;
  std::unique_ptr<Pool> pool_;
  char* ws_ = nullptr;
  char* aux_ = nullptr;
  size_t ws_cap_ = 0, aux_cap_ = 0;
  std::unique_ptr<Regions> wsr_, auxr_;
  std::deque<std::unique_ptr<Request>> waiting_;
  std::vector<std::unique_ptr<Request>> admitted_;
  std::vector<std::unique_ptr<Lane>> active_;
  std::unordered_map<Lane*, Request*> owner_;
  std::vector<Fin> fin_;
  std::vector<hipEvent_t> ev_pool_;
  std::vector<KStat> stats_ = std::vector<KStat>(kNumClasses);
  bool by_b_ = true;
};

#define SCHK(expr)                                                   \
  do {                                                               \
    hipError_t e_ = (expr);                                          \
    if (e_ != hipSuccess)                                            \
      throw Fail{QTX_ERR_HIP, std::string(#expr) + ": " +            \
                                  hipGetErrorString(e_)};            \
  } while (0)

namespace {
constexpr size_t kAuxCap = 64u << 20;        // energies + status words
constexpr int kRoundsPerSegment = 64;
constexpr size_t kSegArena = 8u << 20;
constexpr int kServeStreams = 4;
}  // namespace

Server::Server(qtx_rgf_ctx* c, size_t ws_budget) : c_(c) {
  try {
    SCHK(hipSetDevice(c->device));
    SCHK(hipStreamCreateWithFlags(&s_, hipStreamNonBlocking));
    SCHK(hipStreamCreateWithFlags(&s_read_, hipStreamNonBlocking));
    pool_.reset(new Pool(s_, kServeStreams));
    const char* cp = std::getenv("QTX_SERVE_CLASS");
    by_b_ = !(cp && std::string(cp) == "shape");
    ws_cap_ = ws_budget;
    if (hipMalloc((void**)&ws_, ws_cap_) != hipSuccess) {
      (void)hipGetLastError();
      ws_ = nullptr;
      throw Fail{QTX_ERR_NOMEM};
    }
    aux_cap_ = kAuxCap;
    SCHK(hipMalloc((void**)&aux_, aux_cap_));
    wsr_.reset(new Regions(ws_cap_));
    auxr_.reset(new Regions(aux_cap_));
    th_ = std::thread([this] { loop(); });
  } catch (...) {
    free_resources();              // the destructor does not run for a failed constructor
    throw;
  }
}

void Server::free_resources() {
  pool_.reset();
  for (auto e : ev_pool_) (void)hipEventDestroy(e);
  ev_pool_.clear();
  for (auto& f : fin_) (void)hipEventDestroy(f.ev);
  fin_.clear();
  if (ws_) (void)hipFree(ws_);
  if (aux_) (void)hipFree(aux_);
  if (s_) (void)hipStreamDestroy(s_);
  if (s_read_) (void)hipStreamDestroy(s_read_);
  ws_ = aux_ = nullptr;
  s_ = s_read_ = nullptr;
}

Server::~Server() {
  {
    std::lock_guard<std::mutex> g(mu_);
    stop_ = true;
  }
  cv_in_.notify_all();
  if (th_.joinable()) th_.join();
  free_resources();
}

qtx_status Server::submit(const qtx_rgf_problem& p, uint64_t* ticket) {
  std::unique_ptr<Request> r(new Request());
  r->p = p;
  r->q = make_plan(p);
  if (p.kind == QTX_KIND_G) r->E.assign(p.energies, p.energies + p.n_energies);
  r->p.energies = nullptr;
  if (lane_bytes(r->q, 1) > ws_cap_) return QTX_ERR_NOMEM;
  if ((size_t)p.n_energies * 12 + 1024 > aux_cap_) return QTX_ERR_NOMEM;
  // the largest energy chunk that takes at most half of the workspace, so
  // that other problems can run beside it
  int lo = 1, hi = p.n_energies;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (lane_bytes(r->q, mid) <= ws_cap_ / 2) lo = mid; else hi = mid - 1;
  }
  r->ec_max = lo;
  r->t_sub = Clock::now();
  {
    std::lock_guard<std::mutex> g(mu_);
    if (failed_) return QTX_ERR_HIP;
    r->ticket = next_ticket_++;
    *ticket = r->ticket;
    ++outstanding_;
    incoming_.push_back(std::move(r));
  }
  cv_in_.notify_all();
  return QTX_OK;
}

qtx_status Server::poll(qtx_rgf_completion* out, int cap, int* n, int* pending, int wait_ms) {
  std::unique_lock<std::mutex> g(mu_);
  auto ready = [&] { return !done_.empty() || outstanding_ == 0 || failed_; };
  if (wait_ms < 0) cv_out_.wait(g, ready);
  else if (wait_ms > 0) cv_out_.wait_for(g, std::chrono::milliseconds(wait_ms), ready);
  int k = 0;
  while (k < cap && !done_.empty()) {
    out[k++] = done_.front();
    done_.pop_front();
  }
  *n = k;
  if (pending) *pending = outstanding_;
  return failed_ ? QTX_ERR_HIP : QTX_OK;
}

void Server::admit() {
  while (!waiting_.empty()) {
    Request* r = waiting_.front().get();
    const int ne = r->p.n_energies;
    if (!r->has_aux) {
      const size_t eb = ((size_t)ne * 8 + 255) & ~size_t(255);
      const size_t len = eb + (size_t)ne * 4 + 256;
      size_t off;
      if (!auxr_->alloc(len, &off)) return;
      r->has_aux = true;
      r->aux_off = off;
      r->aux_len = len;
      r->dE = (double*)(aux_ + off);
      r->dinfo = (int*)(aux_ + off + eb);
      if (!r->E.empty()) {
        SCHK(hipMemcpyAsync(r->dE, r->E.data(), sizeof(double) * ne, hipMemcpyHostToDevice, s_read_));
        SCHK(hipStreamSynchronize(s_read_));
      }
    }
    while (r->next_e0 < ne) {
      const int ec = std::min(r->ec_max, ne - r->next_e0);
      const size_t by = lane_bytes(r->q, ec);
      size_t off;
      if (!wsr_->alloc(by, &off)) return;            // wait for memory (arrival order)
      std::unique_ptr<Lane> L(new Lane());
      L->e0 = r->next_e0;
      L->ec = ec;
      L->ws_off = off;
      L->ws_bytes = by;
      r->p.energies = r->E.empty() ? nullptr : r->E.data();
      // requests arrive at any time, so lanes of one class are rarely in
      // phase: classes are kept per block size and spread over the streams
      const uint64_t cls = lane_class(r->q, r->p, by_b_ ? 2 : 0);
      const int xi = pool_->place(cls);
      build_lane(*L, r->p, r->q, ws_ + off, r->next_e0, ec, r->dE, r->dinfo, c_->tuner,
                 pool_->stream(xi));
      L->cls = cls;                    // before add: the pool keys on it
      pool_->add(L.get(), xi);
      owner_[L.get()] = r;
      active_.push_back(std::move(L));
      r->lanes_out++;
      r->next_e0 += ec;
      if (!r->admitted_any) {
        r->admitted_any = true;
        r->t_adm = Clock::now();
      }
    }
    admitted_.push_back(std::move(waiting_.front()));
    waiting_.pop_front();
  }
}

void Server::complete(Request* r) {
  const int ne = r->p.n_energies;
  std::vector<int> info(ne);
  SCHK(hipMemcpyAsync(info.data(), r->dinfo, sizeof(int) * ne, hipMemcpyDeviceToHost, s_read_));
  SCHK(hipStreamSynchronize(s_read_));
  qtx_rgf_completion cm{};
  cm.ticket = r->ticket;
  cm.status = QTX_OK;
  cm.fail_energy = -1;
  cm.fail_block = -1;
  cm.n_energies = ne;
  for (int e = 0; e < ne; ++e)
    if (info[e] != 0) {
      cm.status = info[e] > 0 ? QTX_ERR_SINGULAR : QTX_ERR_NOT_FINITE;
      cm.fail_energy = e;
      cm.fail_block = std::abs(info[e]) - 1;
      break;
    }
  const auto now = Clock::now();
  cm.queue_s = std::chrono::duration<double>(r->t_adm - r->t_sub).count();
  cm.latency_s = std::chrono::duration<double>(now - r->t_sub).count();
  auxr_->release(r->aux_off, r->aux_len);
  for (size_t i = 0; i < admitted_.size(); ++i)
    if (admitted_[i].get() == r) {
      {
        std::lock_guard<std::mutex> g(mu_);
        done_.push_back(cm);
        --outstanding_;
      }
      cv_out_.notify_all();
      admitted_.erase(admitted_.begin() + i);
      return;
    }
}

hipEvent_t Server::get_event() {
  if (!ev_pool_.empty()) {
    hipEvent_t e = ev_pool_.back();
    ev_pool_.pop_back();
    return e;
  }
  hipEvent_t e;
  SCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  return e;
}

// Retire finished lanes whose work has completed; with `block`, wait for
// the oldest one first.
void Server::retire(bool block) {
  if (block && !fin_.empty()) SCHK(hipEventSynchronize(fin_.front().ev));
  for (size_t i = 0; i < fin_.size();) {
    const hipError_t q = hipEventQuery(fin_[i].ev);
    if (q == hipErrorNotReady) {
      ++i;
      continue;
    }
    if (q != hipSuccess) throw Fail{QTX_ERR_HIP};
    Request* r = fin_[i].r;
    ev_pool_.push_back(fin_[i].ev);
    fin_.erase(fin_.begin() + i);
    r->lanes_out--;
    if (r->lanes_out == 0 && r->next_e0 == r->p.n_energies) complete(r);
  }
}

void Server::fail_all(int st) {
  std::lock_guard<std::mutex> g(mu_);
  failed_ = true;
  auto push = [&](Request* r) {
    qtx_rgf_completion cm{};
    cm.ticket = r->ticket;
    cm.status = st;
    cm.fail_energy = -1;
    cm.fail_block = -1;
    cm.n_energies = r->p.n_energies;
    done_.push_back(cm);
  };
  for (auto& r : incoming_) push(r.get());
  for (auto& r : waiting_) push(r.get());
  for (auto& r : admitted_) push(r.get());
  incoming_.clear();
  waiting_.clear();
  admitted_.clear();
  outstanding_ = 0;
  cv_out_.notify_all();
}

void Server::loop() {
  try {
    (void)hipSetDevice(c_->device);
    std::vector<std::pair<Lane*, int>> fin;
    while (true) {
      {
        std::unique_lock<std::mutex> g(mu_);
        if (waiting_.empty() && active_.empty() && fin_.empty() && incoming_.empty()) {
          if (stop_) break;
          cv_in_.wait_for(g, std::chrono::milliseconds(5));
        }
        while (!incoming_.empty()) {
          waiting_.push_back(std::move(incoming_.front()));
          incoming_.pop_front();
        }
      }
      admit();
      if (!pool_->busy()) {
        retire(!fin_.empty());
        continue;
      }
      pool_->step(kSegArena, kRoundsPerSegment, true, false, false, stats_, fin);
      for (auto& f : fin) {
        Lane* l = f.first;
        // its work is queued on its stream: the region may be reused by
        // lanes added later (ordered through the pool's release events)
        wsr_->release(l->ws_off, l->ws_bytes);
        const hipEvent_t ev = get_event();
        SCHK(hipEventRecord(ev, pool_->stream(f.second)));
        fin_.push_back(Fin{ev, owner_[l]});
        owner_.erase(l);
        for (size_t i = 0; i < active_.size(); ++i)
          if (active_[i].get() == l) {
            active_.erase(active_.begin() + i);
            break;
          }
      }
      fin.clear();
      retire(false);
    }
  } catch (const Fail& f) {
    fail_all(f.st);
  } catch (...) {
    fail_all(QTX_ERR_HIP);
  }
}

}  // namespace qtx

using namespace qtx;

qtx_rgf_ctx::qtx_rgf_ctx() = default;
qtx_rgf_ctx::~qtx_rgf_ctx() = default;

void qtx::stop_server(qtx_rgf_ctx* c) { c->server.reset(); }

extern "C" {

qtx_status qtx_rgf_submit(qtx_rgf_ctx* c, const qtx_rgf_problem* p, uint64_t* ticket) {
  if (!c || !p || !ticket) return QTX_ERR_INVALID_ARG;
  const std::string m = validate_problem(*p);
  if (!m.empty()) {
    c->err = "submit: " + m;
    return QTX_ERR_INVALID_ARG;
  }
  try {
    if (!c->server) {
      size_t budget = c->budget;
      if (!budget) {
        size_t fr = 0, tot = 0;
        if (hipSetDevice(c->device) != hipSuccess || hipMemGetInfo(&fr, &tot) != hipSuccess)
          return QTX_ERR_HIP;
        budget = fr / 2;
      }
      c->server.reset(new Server(c, budget));
    }
    return c->server->submit(*p, ticket);
  } catch (const Fail& f) {
    c->err = "request loop could not start" + (f.what.empty() ? std::string() : ": " + f.what);
    return (qtx_status)f.st;
  }
}

qtx_status qtx_rgf_poll(qtx_rgf_ctx* c, qtx_rgf_completion* out, int32_t cap, int32_t* n_out,
                        int32_t* n_pending, int32_t wait_ms) {
  if (!c || !n_out || cap < 0 || (cap > 0 && !out)) return QTX_ERR_INVALID_ARG;
  if (!c->server) {
    *n_out = 0;
    if (n_pending) *n_pending = 0;
    return QTX_OK;
  }
  int n = 0, pend = 0;
  const qtx_status st = c->server->poll(out, cap, &n, &pend, wait_ms);
  *n_out = n;
  if (n_pending) *n_pending = pend;
  return st;
}

}  // extern "C"
