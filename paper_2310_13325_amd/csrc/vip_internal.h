// Internal declarations shared by the translation units of libvip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <string>
#include <vector>

#include "vip.h"

#define VIP_TRY_HIP(expr)                                   \
  do {                                                      \
    hipError_t _e = (expr);                                 \
    if (_e != hipSuccess) {                                 \
      vip::set_last_hip_error(_e, #expr, __FILE__, __LINE__); \
      return VIP_E_HIP;                                     \
    }                                                       \
  } while (0)

#define VIP_TRY(expr)                \
  do {                               \
    vip_status _s = (expr);          \
    if (_s != VIP_OK) return _s;     \
  } while (0)

// Launch bookkeeping: check the launch right after enqueueing it.
#define VIP_LAUNCH_CHECK() VIP_TRY_HIP(hipGetLastError())

namespace vip {

void set_last_hip_error(hipError_t e, const char *expr, const char *file, int line);

constexpr size_t kAlign = 256;
constexpr size_t kStatusBytes = 256;   // status word lives in the first bytes of every workspace

inline size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }

// Bump allocator over a caller workspace: first pass sizes, second pass places.
struct Arena {
  char *base = nullptr;
  size_t used = kStatusBytes;
  template <class T>
  T *take(size_t count) {
    size_t off = align_up(used);
    used = off + count * sizeof(T);
    return base ? reinterpret_cast<T *>(base + off) : nullptr;
  }
  size_t bytes() const { return align_up(used); }
};

inline bool aligned(const void *p) { return (reinterpret_cast<uintptr_t>(p) % kAlign) == 0; }

// Graph cache key: the raw bytes of every argument of a call.
struct KeyBuilder {
  std::string k;
  template <class T>
  KeyBuilder &add(const T &v) {
    k.append(reinterpret_cast<const char *>(&v), sizeof(T));
    return *this;
  }
  KeyBuilder &add_array(const int32_t *p, int32_t n) {
    if (p && n > 0) k.append(reinterpret_cast<const char *>(p), sizeof(int32_t) * size_t(n));
    return *this;
  }
};

}  // namespace vip

struct vip_timing_run {
  hipEvent_t start, stop;
  int kind;
  int64_t launches;
  double point_steps;
};

struct vip_ctx {
  int device = 0;
  int cus = 0;     // compute units of the device
  bool timing = false;
  std::vector<vip_timing_run> runs;     // recorded, not yet read
  std::vector<hipEvent_t> event_pool;   // free events
  hipStream_t user = nullptr;   // caller's stream
  hipStream_t cap = nullptr;    // internal stream for capture / replay
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  bool graph_mode = false;
  int tile = -2;   // step-kernel shape: -2 automatic, -1 one step per launch, >= 0 tile table index
  std::map<std::string, hipGraphExec_t> graphs;
  std::deque<std::string> graph_order;   // cache keys, oldest first
  // Stream the launch helpers enqueue on (user, or cap while capturing).
  hipStream_t s() const { return active; }
  hipStream_t active = nullptr;
};

namespace vip {

// Graphs a context keeps; a new argument set beyond this evicts the oldest.
constexpr size_t kMaxCachedGraphs = 32;

// Runs `body` (a sequence of launches on ctx->s()) either eagerly on the user
// stream or, in graph mode, through a cached hipGraph keyed by `key`.
template <class F>
vip_status run_maybe_graph(vip_ctx *ctx, const std::string &key, F &&body) {
  if (!ctx->graph_mode) {
    ctx->active = ctx->user;
    return body();
  }
  auto it = ctx->graphs.find(key);
  if (it == ctx->graphs.end()) {
    ctx->active = ctx->cap;
    VIP_TRY_HIP(hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal));
    vip_status st = body();
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(ctx->cap, &g);
    ctx->active = ctx->user;
    if (st != VIP_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    VIP_TRY_HIP(e);
    hipGraphExec_t exec = nullptr;
    hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    VIP_TRY_HIP(ei);
    if (ctx->graphs.size() >= kMaxCachedGraphs) {
      // evict the oldest graph once its last replay has finished
      VIP_TRY_HIP(hipStreamSynchronize(ctx->cap));
      auto old = ctx->graphs.find(ctx->graph_order.front());
      (void)hipGraphExecDestroy(old->second);
      ctx->graphs.erase(old);
      ctx->graph_order.pop_front();
    }
    it = ctx->graphs.emplace(key, exec).first;
    ctx->graph_order.push_back(key);
  }
  VIP_TRY_HIP(hipEventRecord(ctx->ev_in, ctx->user));
  VIP_TRY_HIP(hipStreamWaitEvent(ctx->cap, ctx->ev_in, 0));
  VIP_TRY_HIP(hipGraphLaunch(it->second, ctx->cap));
  VIP_TRY_HIP(hipEventRecord(ctx->ev_out, ctx->cap));
  VIP_TRY_HIP(hipStreamWaitEvent(ctx->user, ctx->ev_out, 0));
  return VIP_OK;
}

// Timing of runs of step launches (util.hip).  begin returns -1 when off.
int timing_begin(vip_ctx *ctx, int kind);
void timing_end(vip_ctx *ctx, int run, int64_t launches, double point_steps);

// Device address of the allocation-free step's fixed array on `device`
// (svgd.hip); vip_create calls it with `device` current.
vip_status vip_noalloc_setup(int device);

// Small helpers implemented in util.hip
vip_status fill_u32(hipStream_t s, uint32_t *p, size_t n, uint32_t v);
vip_status fill_f32(hipStream_t s, float *p, size_t n, float v);
vip_status fill_f64(hipStream_t s, double *p, size_t n, double v);
vip_status upload_i32(hipStream_t s, int32_t *dst, const int32_t *host, size_t n);

}  // namespace vip
