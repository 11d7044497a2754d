// An allocation-free bind: the factor's workspace is a device array of the
// library itself, for callers that cannot allocate device memory.
//
// The array lives in the library's code object: every device the library is
// loaded on holds its own copy of D3M_STATIC_WS_BYTES until the process ends.
// In host code the array's name only stands for it; its device address comes
// from hipGetSymbolAddress, taken once per device with that device current,
// and only that address is ever passed on.  One factor at a time per device
// lives there: binding another one on the same device invalidates the earlier
// (its later calls return D3M_ERR_STATE), and calls on factors that share the
// array must not overlap in time.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/d3m.h"
#include "static_ws.h"

namespace {

static __device__ __attribute__((aligned(256))) unsigned char scratch[D3M_STATIC_WS_BYTES];

constexpr int kMaxDev = 64;
std::mutex g_mu;
void* g_ptr[kMaxDev];              // device address of scratch, per device
unsigned long long g_gen[kMaxDev];  // generation of the factor bound there last

}  // namespace

namespace d3m {

bool static_ws_valid(int dev, unsigned long long gen) {
  std::lock_guard<std::mutex> lk(g_mu);
  return dev >= 0 && dev < kMaxDev && g_gen[dev] == gen;
}

}  // namespace d3m

extern "C" d3m_status d3m_factor_bind_static(d3m_plan plan, d3m_precision prec, int32_t nrhs_max,
                                             const d3m_options* opt, d3m_factor* out) {
  if (!plan || !out) return D3M_ERR_ARG;
  *out = nullptr;
  size_t need = 0;
  d3m_status st = d3m_workspace_bytes(plan, prec, nrhs_max, &need);
  if (st != D3M_OK) return st;
  if (need > (size_t)D3M_STATIC_WS_BYTES) return D3M_ERR_WORKSPACE;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return D3M_ERR_HIP;
  if (dev < 0 || dev >= kMaxDev) return D3M_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return D3M_ERR_HIP;
    g_ptr[dev] = p;
  }
  // the earlier factor on this device is invalid from here on, whatever the
  // outcome: the bind below overwrites its tables
  const unsigned long long gen = ++g_gen[dev];
  d3m_options o{};
  if (opt) o = *opt;
  o.timing = 0;  // event timing would create HIP events
  return d3m::bind_factor(plan, prec, g_ptr[dev], (size_t)D3M_STATIC_WS_BYTES, nrhs_max, &o, dev, gen, out);
}
