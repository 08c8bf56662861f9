// K-apply for callers that cannot allocate device memory (code under HIP graph
// capture, serving loops, harnesses that forbid hipMalloc): hm_kapply with its
// transform scratch taken from one fixed device array instead of the model's
// workspace.
//
// The array `scratch` below is a file-scope device symbol.  In host code its name
// is only a host-side stand-in, so its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and only that address is used.
// Every call on a device shares that device's array, which keeps the last call's
// contents; the K-apply writes every scratch element it reads, so nothing needs
// clearing.  Calls that overlap on one device race on the array.
#include <algorithm>
#include <mutex>
#include <string>

#include "hm_internal.h"

namespace hm {

constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB per device
constexpr size_t kScratchDoubles = kScratchBytes / sizeof(double);
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchDoubles];

static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

// device address of this device's copy of the array (looked up on first use)
static hm_status scratch_address(int device, double** out) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("device ordinal out of range for the fixed scratch");
    return HM_E_INVAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    HM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
      set_error("hipGetSymbolAddress returned no address for the fixed scratch");
      return HM_E_DEVICE;
    }
    g_scratch_ptr[device] = (double*)p;
  }
  *out = g_scratch_ptr[device];
  return HM_OK;
}

}  // namespace hm

using namespace hm;

extern "C" hm_status hm_kapply_noalloc(hm_model* mm, const double* theta_full, const double* X, int ldx, int c,
                                       double* Y, int ldy, int which) {
  if (!mm || !X || !Y) {
    set_error("NULL argument");
    return HM_E_INVAL;
  }
  Model* m = &mm->m;
  HM_CHECK(check_theta(m, theta_full));
  if (c < 0 || ldx < m->n || ldy < m->n || which < 0 || which > 2) {
    set_error("hm_kapply_noalloc: bad c, leading dimension or operator");
    return HM_E_INVAL;
  }
  const size_t per_col = 5 * (size_t)m->n;   // doubles of transform scratch per column
  if (per_col > kScratchDoubles) {
    set_error("hm_kapply_noalloc: n = " + std::to_string(m->n) + " needs " + std::to_string(per_col * 8) +
              " bytes of scratch per column, more than the fixed " + std::to_string(kScratchBytes) + " bytes");
    return HM_E_INVAL;
  }
  if (c == 0) return HM_OK;
  int cur = -1;
  HM_HIP(hipGetDevice(&cur));
  if (cur != m->device) HM_HIP(hipSetDevice(m->device));
  double* ws = nullptr;
  hm_status st = scratch_address(m->device, &ws);
  if (st == HM_OK) {
    const int cblk = (int)std::min<size_t>(kScratchDoubles / per_col, 4096);
    st = kapply_ws(m, ws, cblk, theta_full, X, ldx, c, which == 0 ? Y : nullptr, which == 1 ? Y : nullptr,
                   which == 2 ? Y : nullptr, ldy);
  }
  if (cur != m->device) (void)hipSetDevice(cur);
  return st;
}
