// vc_capacitance_static: the capacitance solve of vc_capacitance with every device array
// of the solve taken from one fixed-size static device array instead of allocations, for
// callers that cannot allocate device memory.
//
// The array `scratch` below is a device symbol: in host code its name is a host-side
// stand-in, not a device address.  Each device's address of its own copy is looked up
// once (hipGetSymbolAddress with that device current) and kept in scratch_base[device];
// only that address is ever passed to kernels or copies.
#include <cstring>
#include <mutex>

#include "mvp_kernels.h"
#include "problem.h"
#include "solver.h"

namespace {

// VC_STATIC_SCRATCH_BYTES of include/voxcap.h
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* scratch_base[kMaxDevices] = {};

// device address of `scratch` on `dev` (which must be the current device)
vc_status scratch_address(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) {
    vc::set_error("device ordinal %d beyond the %d the static scratch table covers", dev, kMaxDevices);
    return VC_ERR_ARG;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!scratch_base[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      vc::set_error("hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
      return VC_ERR_HIP;
    }
    scratch_base[dev] = static_cast<char*>(p);
  }
  *out = scratch_base[dev];
  return VC_OK;
}

}  // namespace

using namespace vc;

extern "C" vc_status vc_capacitance_static(vc_problem* p, const vc_solve_opts* opts, double* C, double* rho_dev,
                                           vc_stats* stats, void* hip_stream) {
  if (!p) { set_error("null problem"); return VC_ERR_ARG; }
  if (p->hip_failed) { set_error("problem unusable after a HIP error"); return VC_ERR_HIP; }
  if (p->pack) { set_error("packed sets are solved by vc_pack_capacitance"); return VC_ERR_ARG; }
  vc_solve_opts o;
  vc_status s = capacitance_check(p, opts, C, &o);
  if (s != VC_OK) return s;
  if (o.use_precond == 3) {
    set_error("use_precond 3 builds its blocks (allocates) on first use; not available without allocation");
    return VC_ERR_ARG;
  }
  const int64_t N = npanels(p);
  const size_t need = solve_ws_layout(N, p->m, o.restart, nullptr, nullptr);
  if (need > kScratchBytes) {
    set_error("this solve needs %zu bytes of scratch (N=%lld, m=%d, restart %d); the static array holds %zu",
              need, (long long)N, p->m, o.restart, kScratchBytes);
    return VC_ERR_ARG;
  }
  const hipError_t ed = hipSetDevice(p->device);
  if (ed != hipSuccess) { set_error("hipSetDevice: %s", hipGetErrorString(ed)); return VC_ERR_HIP; }
  char* base = nullptr;
  s = scratch_address(p->device, &base);
  if (s != VC_OK) return s;
  const double t0 = now_s();
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  SolveWs ws;
  solve_ws_layout(N, p->m, o.restart, base, &ws);
  // the Gram-Schmidt completion counters rest at zero between launches: clear them in
  // case an earlier call stopped part-way (a fill kernel, no memset node)
  hipError_t e = launch_zero_u32(ws.cnt, cgs_counter_size(o.restart + 1, p->m), st);
  if (e != hipSuccess) {
    set_error("clearing the scratch counters: %s", hipGetErrorString(e));
    p->hip_failed = true;
    return VC_ERR_HIP;
  }
  const SolveWs own = p->ws;   // the problem's own regions (captured graphs point there)
  p->ws = ws;
  p->ws_static = true;
  s = capacitance_run(p, o, C, rho_dev, stats, st, nullptr, t0);
  p->ws = own;
  p->ws_static = false;
  if (s == VC_ERR_HIP) p->hip_failed = true;
  return s;
}
