// Error reporting and workspace sizing for the C ABI.
#include <cstdarg>
#include <cstdio>

#include "common.hpp"
#include "layout.hpp"

namespace mds {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

int fail(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

int check_launch(const char *what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MD_EHIP, "%s: %s", what, hipGetErrorString(e));
  return MD_OK;
}

size_t lds_limit() {
  static size_t cache[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 65536 - 4096;
  if (cache[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        v < 65536)
      v = 65536;
    cache[dev] = size_t(v) - 4096;
  }
  return cache[dev];
}

}  // namespace mds

extern "C" size_t md_device_lds_bytes(void) { return mds::lds_limit(); }

extern "C" const char *md_last_error(void) { return mds::g_err; }

extern "C" size_t md_workspace_bytes(int fn, int m, int N, int n, int d, int M, int max_deg) {
  if (fn == MD_FN_PADE) {  // N: denominator degree, n: numerator degree, M: series count
    if (!mds::valid_m(m) || N < 0 || N > 64 || n < 0 || M < 0) return 0;
    return mds::PadeLayout(m, N, M).bytes;
  }
  if (!mds::valid_m(m) || N < 1 || n < 1 || d < 0 || M < 0 || max_deg < 0) return 0;
  switch (fn) {
    case MD_FN_EVAL: return mds::EvalLayout(m, N, n, d, M, max_deg).bytes;
    case MD_FN_SOLVE: return mds::SolveLayout(m, N, n, d).bytes;
    case MD_FN_NEWTON: return mds::NewtonLayout(m, N, n, d, M, max_deg).bytes;
    case MD_FN_ADJOINT: return mds::AdjointLayout(m, N, n, d, M, max_deg, false).bytes;
    case MD_FN_ADJOINT_STORE: return mds::AdjointLayout(m, N, n, d, M, max_deg, true).bytes;
    case MD_FN_PROTOCOL: return mds::ProtocolLayout(m, N, n, d, M, max_deg).bytes;
    case MD_FN_PADE: return mds::PadeLayout(m, N, M).bytes;
    default: return 0;
  }
}
