// Context of the RGF library (shared by the C ABI and the serving loop).
#pragma once
#include <condition_variable>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/qtx_rgf.h"
#include "exec.h"

namespace qtx {
class Server;
}

struct qtx_rgf_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  uint64_t budget = 0;
  uint32_t flags = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  char* aux = nullptr;
  size_t aux_bytes = 0;
  std::string err;
  std::vector<qtx::KStat> stats = std::vector<qtx::KStat>(qtx::kNumClasses);
  std::unique_ptr<qtx::Pool> pool;       // executors on the context's streams
  qtx::Tuner tuner;
  bool graphs = true;
  int batch_size_key = 2;                // lane classes of a batch (lane_class)
  int split = 1;                         // energy chunks per large problem, one stream each
  bool busy = false;
  std::unique_ptr<qtx::Server> server;   // request loop (qtx_rgf_submit)
  // defined with the request loop, where Server is complete
  qtx_rgf_ctx();
  ~qtx_rgf_ctx();
};


namespace qtx {

#define HIPCHK(ctx, expr)                                                    \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess) {                                                  \
      (ctx)->err = std::string(#expr) + ": " + hipGetErrorString(e_);        \
      throw Fail{QTX_ERR_HIP};                                               \
    }                                                                        \
  } while (0)

// First-fit allocator over [0, cap) with 256-byte granularity.
class Regions {
 public:
  explicit Regions(size_t cap) { free_[0] = cap; }
  bool alloc(size_t bytes, size_t* off) {
    bytes = (bytes + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t o = it->first + bytes;
        free_.erase(it);
        if (rest) free_[o] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;
};

// Argument checks shared by qtx_rgf_solve_batch and qtx_rgf_submit; returns
// an error message or an empty string.
std::string validate_problem(const qtx_rgf_problem& p);

constexpr size_t kArenaLimit = 32u << 20;    // descriptor bytes per segment

// Workspace budget of a call: the context's, else 90% of the free memory
// plus what the context already holds.
size_t budget_now(qtx_rgf_ctx* c);
// Grow-only device buffer *p of *have bytes to at least `need` bytes (the
// pool is drained and its graphs released first); QTX_ERR_NOMEM on failure.
void ensure(qtx_rgf_ctx* c, char** p, size_t* have, size_t need);
// Run lanes to completion in merged launches on the pool's first stream.
void run_lanes_to_end(qtx_rgf_ctx* c, std::vector<Lane*>& lanes);

// Drain and stop the context's request loop, if it was started.
void stop_server(qtx_rgf_ctx* c);

// Resolve, once per device and with that device current, the address of the
// static scratch array of qtx_rgf_zinv_noalloc.
hipError_t noalloc_init(int device);
// Scratch bytes qtx_rgf_zinv_noalloc needs for `batch` matrices of size b.
size_t noalloc_work_bytes(int b, int batch);

}  // namespace qtx
