// stm_match_noalloc: the exact matching of stm_match on a fixed device array
// instead of allocated scratch, for callers that cannot allocate device memory.
//
// The array `scratch` below holds every buffer the matching's kernels need
// besides the caller's inputs and outputs: the validation words, the frame
// index, the model angles, the unary table, the BF16 copies (split precision)
// and, for as many offsets at a time as fit, the recursion's value tables,
// last state pairs and degenerate flags.  Its device address is looked up
// once per device at context creation (hipGetSymbolAddress, with the device
// current) and only that address is handed to kernels: in host code the
// array's name is a host-side stand-in, not a device address.
//
// Every call on a device shares that device's array, which keeps the last
// call's contents; nothing in it has to start at zero except the validation
// words, which a fill kernel clears at the start of each call.  Calls that
// overlap on one device (from several threads, or queued on different streams
// without ordering) race on the array.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "host_common.h"

static __device__ __align__(256) unsigned char scratch[STM_NOALLOC_SCRATCH_BYTES];

namespace {

// Device address of `scratch` per HIP device (null until looked up or when the
// lookup failed; the failure's message is kept for the entry point).
constexpr int kMaxDevices = 64;
std::mutex g_mu;
bool g_done[kMaxDevices] = {};
unsigned char* g_ptr[kMaxDevices] = {};
std::string g_msg[kMaxDevices];

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Carves consecutive 256-byte aligned pieces out of the array.
struct Carver {
  unsigned char* base;
  size_t used = 0;
  template <class T>
  T* take(size_t count) {
    T* p = reinterpret_cast<T*>(base + used);
    used += align256(count * sizeof(T));
    return p;
  }
};

}  // namespace

namespace stmh {

// Looks up the array's device address on `device` (the current device), once
// per device.  Returns STM_OK or STM_EHIP; a failure is remembered and
// reported by stm_match_noalloc, not by the caller.
int noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return STM_OK;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_done[device]) return STM_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  g_done[device] = true;
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    g_ptr[device] = nullptr;
    g_msg[device] = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    return STM_EHIP;
  }
  g_ptr[device] = static_cast<unsigned char*>(p);
  return STM_OK;
}

}  // namespace stmh

using namespace stmh;

extern "C" int stm_match_noalloc(stm_ctx* ctx, const stm_points* model, const stm_points* scene,
                                 const stm_params* params, int32_t tau_begin, int32_t tau_end,
                                 float* energy32, double* energy64, double* energy_u64, int32_t* assign,
                                 void* hip_stream) {
  err().clear();
  if (!ctx) return fail(STM_EINVAL, "null context");
  if (!params) return fail(STM_EINVAL, "null params");
  if (!(params->flags & STM_DEVICE_PTRS))
    return fail(STM_EINVAL, "stm_match_noalloc takes device pointers only (STM_DEVICE_PTRS)");
  if (ctx->device < 0 || ctx->device >= kMaxDevices) return fail(STM_EUNSUPPORTED, "device index above 63");
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_done[ctx->device]) return fail(STM_EHIP, "scratch array not looked up for this device");
    if (!g_ptr[ctx->device]) return fail(STM_EHIP, g_msg[ctx->device]);
    base = g_ptr[ctx->device];
  }
  int rc = check_shapes(model, scene, params);
  if (rc) return rc;
  const int M = model->n, S = scene->n, F = scene->n_frames, dim = model->dim;
  const bool bf16 = (params->flags & STM_UNARY_BF16) != 0;

  // the fixed part of the layout, checked against the array before any work
  Carver cv{base};
  FixedPrep fp;
  fp.val = cv.take<int32_t>(2);
  fp.fstart = cv.take<int32_t>((size_t)F + 1);
  MatchScratch sc;
  sc.theta = cv.take<float2>(M);
  sc.U = cv.take<float>((size_t)M * S);
  if (bf16) {
    const int Mp = bf16_rows_model(M), Sp = bf16_rows_scene(S), dp = stm::bf16_padded_dim(dim);
    sc.bf.fb = cv.take<uint16_t>((size_t)Mp * dp);
    sc.bf.fn = cv.take<float>(Mp);
    sc.bf.gb = cv.take<uint16_t>((size_t)Sp * dp);
    sc.bf.gn = cv.take<float>(Sp);
  }
  const size_t per_tau = vt_bytes_per_offset(M, params) + sizeof(int2) + sizeof(int32_t);
  const size_t limit = STM_NOALLOC_SCRATCH_BYTES;
  // three more alignment paddings for the per-offset buffers
  if (cv.used + per_tau + 3 * 256 > limit)
    return fail(STM_EINVAL, "inputs need " + std::to_string(cv.used + per_tau + 3 * 256) +
                                " bytes of scratch for one offset, above the fixed " + std::to_string(limit) +
                                " bytes (STM_NOALLOC_SCRATCH_BYTES)");

  Prepared pr;
  if ((rc = prepare(ctx, model, scene, params, hip_stream, pr, &fp))) return rc;
  if ((rc = check_range(pr, tau_begin, tau_end))) return rc;
  const int n_tau = tau_end - tau_begin;
  if (n_tau == 0) return STM_OK;
  if (!energy32 || !assign) return fail(STM_EINVAL, "energy32 and assign are required");

  // as many offsets per chunk as the rest of the array holds
  const size_t rest = limit - cv.used - 3 * 256;
  sc.chunk = static_cast<int>(std::min<size_t>((size_t)n_tau, rest / per_tau));
  sc.last2 = cv.take<int2>(sc.chunk);
  sc.degen = cv.take<int32_t>(sc.chunk);
  sc.vt = cv.take<float>(vt_bytes_per_offset(M, params) / sizeof(float) * sc.chunk);
  if (cv.used > limit) return fail(STM_EINVAL, "scratch layout exceeds the fixed array");
  return match_kernels(ctx, pr, params, tau_begin, n_tau, energy32, energy64, energy_u64, assign, sc, false);
}
