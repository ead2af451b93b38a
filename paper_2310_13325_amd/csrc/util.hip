// Context management, status handling, fills, small uploads, the Ricker
// wavelet and Philox normals.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "vip_internal.h"
#include "philox.h"

namespace vip {

static thread_local char g_last_error[512] = {0};

void set_last_hip_error(hipError_t e, const char *expr, const char *file, int line) {
  std::snprintf(g_last_error, sizeof(g_last_error), "%s (%d) in %s at %s:%d", hipGetErrorString(e),
                int(e), expr, file, line);
}

template <class T>
__global__ void fill_kernel(T *p, size_t n, T v) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  size_t stride = size_t(gridDim.x) * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

template <class T>
static vip_status fill(hipStream_t s, T *p, size_t n, T v) {
  if (n == 0) return VIP_OK;
  size_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  fill_kernel<T><<<dim3(unsigned(blocks)), dim3(256), 0, s>>>(p, n, v);
  VIP_LAUNCH_CHECK();
  return VIP_OK;
}

vip_status fill_u32(hipStream_t s, uint32_t *p, size_t n, uint32_t v) { return fill(s, p, n, v); }
vip_status fill_f32(hipStream_t s, float *p, size_t n, float v) { return fill(s, p, n, v); }
vip_status fill_f64(hipStream_t s, double *p, size_t n, double v) { return fill(s, p, n, v); }

// Host values travel as kernel arguments, so uploads need no pinned staging
// buffer, no allocation and stay valid under stream capture.
constexpr int kUploadChunk = 960;
struct UploadChunk {
  int32_t v[kUploadChunk];
};

__global__ void upload_kernel(int32_t *dst, UploadChunk c, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = c.v[i];
}

vip_status upload_i32(hipStream_t s, int32_t *dst, const int32_t *host, size_t n) {
  for (size_t off = 0; off < n; off += kUploadChunk) {
    int m = int(n - off < size_t(kUploadChunk) ? n - off : size_t(kUploadChunk));
    UploadChunk c;
    std::memcpy(c.v, host + off, sizeof(int32_t) * size_t(m));
    upload_kernel<<<dim3((m + 255) / 256), dim3(256), 0, s>>>(dst + off, c, m);
    VIP_LAUNCH_CHECK();
  }
  return VIP_OK;
}

__global__ void ricker_kernel(float *out, int nt, double dt, double f0, double t0) {
  int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nt) return;
  double t = double(n) * dt - t0;
  double a = M_PI * f0 * t;
  a *= a;
  out[n] = float((1.0 - 2.0 * a) * exp(-a));
}

__global__ void philox_normals_kernel(float *out, int64_t count, uint32_t k0, uint32_t k1,
                                      uint32_t s0, uint32_t s1) {
  int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (4 * q >= count) return;
  float z[4];
  philox_normals4(uint64_t(q), k0, k1, s0, s1, z);
  for (int k = 0; k < 4; ++k)
    if (4 * q + k < count) out[4 * q + k] = z[k];
}

__global__ void philox_words_kernel(uint32_t *out, int64_t nblocks, uint32_t k0, uint32_t k1,
                                    uint32_t s0, uint32_t s1) {
  int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= nblocks) return;
  uint32_t c[4] = {uint32_t(q), uint32_t(uint64_t(q) >> 32), s0, s1};
  philox4x32_10(c, k0, k1);
  for (int w = 0; w < 4; ++w) out[4 * q + w] = c[w];
}

static hipEvent_t take_event(vip_ctx *ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

int timing_begin(vip_ctx *ctx, int kind) {
  if (!ctx->timing || ctx->active != ctx->user) return -1;
  vip_timing_run r;
  r.start = take_event(ctx);
  r.stop = take_event(ctx);
  if (!r.start || !r.stop) return -1;
  r.kind = kind;
  r.launches = 0;
  r.point_steps = 0.0;
  if (hipEventRecord(r.start, ctx->active) != hipSuccess) return -1;
  ctx->runs.push_back(r);
  return int(ctx->runs.size()) - 1;
}

void timing_end(vip_ctx *ctx, int run, int64_t launches, double point_steps) {
  if (run < 0) return;
  vip_timing_run &r = ctx->runs[size_t(run)];
  r.launches = launches;
  r.point_steps = point_steps;
  (void)hipEventRecord(r.stop, ctx->active);
}

}  // namespace vip

using namespace vip;

extern "C" {

const char *vip_status_string(int status) {
  switch (status) {
    case VIP_OK: return "VIP_OK";
    case VIP_E_ARG: return "VIP_E_ARG: invalid argument";
    case VIP_E_CFL: return "VIP_E_CFL: time step above the stability limit";
    case VIP_E_WORKSPACE: return "VIP_E_WORKSPACE: workspace too small or misaligned";
    case VIP_E_HIP: return g_last_error[0] ? g_last_error : "VIP_E_HIP: HIP runtime error";
    case VIP_E_NOT_PD: return "VIP_E_NOT_PD: kernel matrix not positive definite";
    case VIP_E_NONFINITE: return "VIP_E_NONFINITE: non-finite value on the device";
    case VIP_E_UNSUPPORTED: return "VIP_E_UNSUPPORTED: option not implemented";
    case VIP_E_SCRATCH:
      return "VIP_E_SCRATCH: the step needs more than the VIP_NOALLOC_SCRATCH_BYTES (64 MiB) "
             "fixed array of vip_svgd_step_noalloc; use vip_svgd_step with a workspace";
    default: return "unknown vip_status";
  }
}

int vip_version(void) { return 10000; }

vip_status vip_create(vip_ctx **out, int device, void *stream) {
  if (!out) return VIP_E_ARG;
  *out = nullptr;
  int count = 0;
  VIP_TRY_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return VIP_E_ARG;
  VIP_TRY_HIP(hipSetDevice(device));
  VIP_TRY(vip_noalloc_setup(device));
  int cus = 0;
  VIP_TRY_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
  vip_ctx *ctx = new vip_ctx();
  ctx->device = device;
  ctx->cus = cus;
  ctx->user = static_cast<hipStream_t>(stream);
  ctx->active = ctx->user;
  hipError_t e = hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_out, hipEventDisableTiming);
  if (e != hipSuccess) {
    set_last_hip_error(e, "vip_create", __FILE__, __LINE__);
    delete ctx;
    return VIP_E_HIP;
  }
  *out = ctx;
  return VIP_OK;
}

vip_status vip_destroy(vip_ctx *ctx) {
  if (!ctx) return VIP_E_ARG;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->user);
  (void)hipStreamSynchronize(ctx->cap);
  for (auto &kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto &r : ctx->runs) {
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
  if (ctx->ev_in) (void)hipEventDestroy(ctx->ev_in);
  if (ctx->ev_out) (void)hipEventDestroy(ctx->ev_out);
  if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
  delete ctx;
  return VIP_OK;
}

vip_status vip_set_stream(vip_ctx *ctx, void *stream) {
  if (!ctx) return VIP_E_ARG;
  ctx->user = static_cast<hipStream_t>(stream);
  ctx->active = ctx->user;
  return VIP_OK;
}

vip_status vip_set_graph_mode(vip_ctx *ctx, int enable) {
  if (!ctx) return VIP_E_ARG;
  ctx->graph_mode = enable != 0;
  return VIP_OK;
}

vip_status vip_set_timing(vip_ctx *ctx, int enable) {
  if (!ctx) return VIP_E_ARG;
  ctx->timing = enable != 0;
  return VIP_OK;
}

vip_status vip_read_timing(vip_ctx *ctx, vip_timing *out) {
  if (!ctx || !out) return VIP_E_ARG;
  std::memset(out, 0, sizeof(*out));
  VIP_TRY_HIP(hipSetDevice(ctx->device));
  VIP_TRY_HIP(hipStreamSynchronize(ctx->user));
  for (auto &r : ctx->runs) {
    float ms = 0.0f;
    VIP_TRY_HIP(hipEventElapsedTime(&ms, r.start, r.stop));
    if (r.kind >= 0 && r.kind < VIP_TIMING_KINDS) {
      out->launches[r.kind] += r.launches;
      out->ms[r.kind] += double(ms);
      out->point_steps[r.kind] += r.point_steps;
    }
    ctx->event_pool.push_back(r.start);
    ctx->event_pool.push_back(r.stop);
  }
  ctx->runs.clear();
  return VIP_OK;
}

vip_status vip_poll(vip_ctx *ctx, void *ws, uint32_t *flags) {
  if (!ctx || !ws || !flags) return VIP_E_ARG;
  VIP_TRY_HIP(hipSetDevice(ctx->device));
  VIP_TRY_HIP(hipStreamSynchronize(ctx->user));
  uint32_t v = 0;
  VIP_TRY_HIP(hipMemcpy(&v, ws, sizeof(v), hipMemcpyDeviceToHost));
  *flags = v;
  uint32_t zero = 0;
  VIP_TRY_HIP(hipMemcpy(ws, &zero, sizeof(zero), hipMemcpyHostToDevice));
  return VIP_OK;
}

vip_status vip_ricker(vip_ctx *ctx, int32_t nt, double dt, double f0, double t0, float *out) {
  if (!ctx || !out || nt <= 0 || !(dt > 0.0) || !(f0 > 0.0)) return VIP_E_ARG;
  if (!(t0 > 0.0)) t0 = 1.5 / f0;
  VIP_TRY_HIP(hipSetDevice(ctx->device));
  ricker_kernel<<<dim3((nt + 255) / 256), dim3(256), 0, ctx->user>>>(out, nt, dt, f0, t0);
  VIP_LAUNCH_CHECK();
  return VIP_OK;
}

vip_status vip_philox_normals(vip_ctx *ctx, int64_t count, uint64_t seed, uint64_t stream,
                              float *out) {
  if (!ctx || !out || count < 0) return VIP_E_ARG;
  if (count == 0) return VIP_OK;
  VIP_TRY_HIP(hipSetDevice(ctx->device));
  int64_t quads = (count + 3) / 4;
  philox_normals_kernel<<<dim3(unsigned((quads + 255) / 256)), dim3(256), 0, ctx->user>>>(
      out, count, uint32_t(seed), uint32_t(seed >> 32), uint32_t(stream), uint32_t(stream >> 32));
  VIP_LAUNCH_CHECK();
  return VIP_OK;
}

vip_status vip_philox_uint32(vip_ctx *ctx, int64_t nblocks, uint64_t seed, uint64_t stream,
                             uint32_t *out) {
  if (!ctx || !out || nblocks < 0) return VIP_E_ARG;
  if (nblocks == 0) return VIP_OK;
  VIP_TRY_HIP(hipSetDevice(ctx->device));
  philox_words_kernel<<<dim3(unsigned((nblocks + 255) / 256)), dim3(256), 0, ctx->user>>>(
      out, nblocks, uint32_t(seed), uint32_t(seed >> 32), uint32_t(stream), uint32_t(stream >> 32));
  VIP_LAUNCH_CHECK();
  return VIP_OK;
}

}  // extern "C"
