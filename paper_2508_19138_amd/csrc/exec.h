// Host runtime of the RGF library: the operation stream of one solve lane,
// the merged-launch scheduler, the descriptor arena, graph replay and the
// tile autotuner.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "qtx_internal.h"

namespace qtx {

constexpr int kClassZgemm = 0, kClassCgemm = 1, kClassInv = 2, kClassElem = 3;
constexpr int kNumClasses = 4;

struct KStat {
  int64_t launches = 0;
  double ms = 0, flops = 0, bytes = 0;
};

enum class OpK : uint8_t { Gemm, Inv, Lin, Trans };

// One step of one lane: up to a few independent descriptors of one kind
// that are issued together (they may share a launch with other lanes').
struct Op {
  OpK k = OpK::Gemm;
  char opa = 'N', opb = 'N';
  bool fp32 = false;
  int cfg = 0;
  int first = 0, count = 0;   // range in the lane's descriptor table of kind k
  double flops = 0, bytes = 0;
};

// A lane is an independent solve: one problem restricted to a contiguous
// chunk of its energies, with its own workspace region.  Its operations are
// executed in order; different lanes are independent.
struct Lane {
  std::vector<Op> ops;
  std::vector<GemmDesc> gd;
  std::vector<InvDesc> id;
  std::vector<LinCombDesc> ld;
  std::vector<TransDesc> td;
  size_t next = 0;
  int problem = -1;
  int e0 = 0, ec = 0;
  size_t ws_off = 0, ws_bytes = 0;
  uint64_t cls = 0;          // shape class (lanes of one class run in lockstep)
  double work = 0;           // flops of all its operations
  bool done() const { return next >= ops.size(); }
};

// Thrown for HIP failures; carries the status for the ABI.
struct Fail {
  int st;
  std::string what = {};     // the failing call, when one is known
};

class Tuner {
 public:
  // Tile configuration for complex products of shape M x N x K.
  int cfg(int M, int N, int K, bool fp32, hipStream_t s);
  void set_enabled(bool on) { enabled_ = on; }
  std::string cache_path() const;

 private:
  int measure(int b, bool fp32, hipStream_t s);
  void load();
  void save() const;
  std::mutex mu_;            // the request loop and callers share the tuner
  bool loaded_ = false;
  bool enabled_ = true;
  std::map<std::string, int> table_;
};

// One kernel launch of a merged schedule.
struct LaunchRec {
  enum Kind : uint8_t { Gemm, Panel, Gather, Permute, Lin, Trans, TallSelect, TallFinal, TallApply,
                        Small } kind;
  char opa, opb;
  bool fp32;
  int cfg;        // gemm tile config, rows per thread R (Panel, Small) or width W (Gather)
  int k0;         // Panel
  size_t desc_off, prefix_off;
  int nd, total;
  int cls;
  double flops, bytes;
};

class Executor {
 public:
  explicit Executor(hipStream_t s) : s_(s) {}
  ~Executor();
  // Advance the lanes by merged rounds until every lane is done or the
  // arena limit is reached; returns the number of rounds emitted.  The
  // caller then calls flush() to upload and launch.
  // A segment also ends after the round in which it reaches max_launches.
  int build(std::vector<Lane*>& lanes, size_t arena_limit, int max_rounds = 1 << 30,
            bool stop_on_finish = false, int max_launches = 1 << 30);
  // Upload and launch what build() produced (graph replay when the same
  // segment was seen before and graphs are enabled).
  void flush(bool profile, bool graphs, std::vector<KStat>& stats);
  void sync_and_collect(std::vector<KStat>& stats);
  bool empty() const { return recs_.empty(); }
  void release();
  // The arena slot the next eager flush uses is free (no wait needed).
  bool slot_ready() const;
  void wait_slot();
  hipStream_t stream() const { return s_; }

 private:
  template <class D>
  size_t put(const std::vector<D>& v);
  size_t put_prefix(const std::vector<int>& p);
  void emit_group(std::vector<std::pair<Lane*, Op*>>& ops);
  void issue(char* dev_arena, bool profile);

  hipStream_t s_;
  std::vector<char> host_;          // arena being built
  std::vector<LaunchRec> recs_;
  // double-buffered device / pinned arenas
  char* dev_[2] = {nullptr, nullptr};
  size_t dev_cap_[2] = {0, 0};
  char* pin_[2] = {nullptr, nullptr};
  size_t pin_cap_[2] = {0, 0};
  hipEvent_t done_[2] = {nullptr, nullptr};
  int slot_ = 0;
  // profiling
  struct Pending { int cls; hipEvent_t a, b; double flops, bytes; };
  std::vector<Pending> pending_;
  std::vector<hipEvent_t> ev_pool_;
  // graph cache
  struct GraphEntry { hipGraphExec_t exec; char* arena; size_t bytes; uint64_t last; };
  std::unordered_map<uint64_t, GraphEntry> graphs_;
  std::unordered_map<uint64_t, int> seen_;
  uint64_t tick_ = 0;
  hipEvent_t get_event();
};

// Executors on several streams advancing disjoint sets of lanes.  Lanes of
// one shape class go to the same executor, where they run in lockstep and
// share launches; different classes overlap on the device.  A lane whose
// workspace region was used by a lane of another executor is ordered after
// it through that executor's release event.
constexpr int kPoolSegLaunches = 256;

class Pool {
 public:
  Pool(hipStream_t main, int n_streams);   // stream 0 is `main` (not owned)
  ~Pool();
  int size() const { return (int)x_.size(); }
  hipStream_t stream(int x) const { return x_[x].s; }
  Executor& exe(int x) { return *x_[x].exe; }
  // Executor for a new lane of class `cls` (lanes keep it in l->cls).
  int place(uint64_t cls);
  // Lane l (already built) joins executor x; x's stream first waits for
  // the region releases recorded by the other executors.
  void add(Lane* l, int x);
  // Issue one segment on every executor that has lanes and a free arena
  // slot (if none has, wait for one first).  Lanes that finished are
  // appended to `done` with their executor; their work is queued, and
  // their regions may be given to lanes added afterwards.  While several
  // executors have lanes, segments are cut at kPoolSegLaunches launches:
  // one host thread feeds every stream, and a long segment would hold it
  // in the launch calls of one stream (whose hardware queue is full) while
  // the other streams run dry.
  void step(size_t arena_limit, int max_rounds, bool stop_on_finish, bool profile,
            bool graphs, std::vector<KStat>& stats, std::vector<std::pair<Lane*, int>>& done);
  bool busy() const;
  void fork();        // every stream waits for the work queued on stream 0
  void join();        // stream 0 waits for the work queued on the others
  void sync_and_collect(std::vector<KStat>& stats);
  void sync();
  void release();     // graphs and arenas of every executor

 private:
  void destroy();
  struct X {
    std::unique_ptr<Executor> exe;
    hipStream_t s = nullptr;
    bool own = false;
    std::vector<Lane*> lanes;
    double load = 0;
    hipEvent_t rel = nullptr;        // recorded after lanes finished
    uint64_t rel_count = 0;
    std::vector<uint64_t> waited;    // rel_count of each other executor seen
    hipEvent_t ev = nullptr;         // fork/join
  };
  std::vector<X> x_;
  std::map<uint64_t, int> cls_x_;    // class -> executor while it has lanes
  std::map<uint64_t, int> cls_n_;
};

}  // namespace qtx
