// marfa_io.hip -- PT-table record files (Appendix A of the paper): one
// direct-access binary file per layer, records of 20481 single-precision
// values, record r covering [10 r, 10 r + 10] cm^-1 at byte offset
// (r - 1) * 20481 * 4.  Host code only.
#include <hip/hip_runtime.h>

#include <fcntl.h>
#include <unistd.h>

#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "marfa.h"
#include "marfa_internal.h"

namespace {

constexpr int64_t kStep = 20480;              // lattice steps per 10 cm^-1 record interval
constexpr int64_t kNT = MARFA_PTBIN_NT;       // values per record (both ends)
constexpr int64_t kBatch = 128;               // records per host buffer (10.5 MB)

int64_t floor_div(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

marfa_status io_fail(const char* what, const char* path) {
  char buf[512];
  std::snprintf(buf, sizeof buf, "%s %s: %s", what, path, std::strerror(errno));
  return marfa::marfa_set_error(MARFA_E_IO, buf);
}

bool write_all(int fd, const char* p, size_t n, off_t off) {
  while (n > 0) {
    const ssize_t w = pwrite(fd, p, n, off);
    if (w < 0) {
      if (errno == EINTR) continue;
      return false;
    }
    p += w;
    n -= (size_t)w;
    off += w;
  }
  return true;
}

}  // namespace

using marfa::marfa_set_error;

extern "C" marfa_status marfa_ptbin_write(const char* path, const float* values, int64_t n_points, double nu_begin,
                                          int32_t values_on_device, void* hip_stream, int32_t flags,
                                          int32_t* records_written) {
  if (records_written) *records_written = 0;
  if (!path) return marfa_set_error(MARFA_E_INVALID, "ptbin: null path");
  if (n_points < 0) return marfa_set_error(MARFA_E_INVALID, "ptbin: negative n_points");
  if (n_points > 0 && !values) return marfa_set_error(MARFA_E_INVALID, "ptbin: null values");
  if (flags & ~MARFA_PTBIN_TRUNCATE) return marfa_set_error(MARFA_E_INVALID, "ptbin: unknown flags");
  if (!std::isfinite(nu_begin) || nu_begin < 0.0 || nu_begin * 2048.0 > 9.0e15)
    return marfa_set_error(MARFA_E_INVALID, "ptbin: nu_begin must be finite and >= 0");
  const double mb = nu_begin * 2048.0;
  const double mr = std::nearbyint(mb);
  if (std::fabs(mb - mr) > 1e-6) return marfa_set_error(MARFA_E_INVALID, "ptbin: nu_begin is not on the 2^-11 lattice");
  const int64_t m0 = (int64_t)mr;
  // whole record intervals inside [m0, m0 + n_points - 1]
  const int64_t r_lo = std::max<int64_t>(1, floor_div(m0 + kStep - 1, kStep));
  const int64_t r_hi = n_points > 0 ? floor_div(m0 + n_points - 1 - kStep, kStep) : r_lo - 1;
  if (r_hi - r_lo + 1 > (int64_t)INT32_MAX) return marfa_set_error(MARFA_E_INVALID, "ptbin: too many records");

  const int fd = open(path, O_WRONLY | O_CREAT | ((flags & MARFA_PTBIN_TRUNCATE) ? O_TRUNC : 0), 0644);
  if (fd < 0) return io_fail("ptbin: cannot open", path);
  marfa_status st = MARFA_OK;
  std::vector<float> stage, rec;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  int64_t done = 0;
  for (int64_t r0 = r_lo; r0 <= r_hi && st == MARFA_OK; r0 += kBatch) {
    const int64_t nb = std::min<int64_t>(kBatch, r_hi - r0 + 1);
    const int64_t first = r0 * kStep - m0;        // source index of the batch's first value
    const int64_t count = nb * kStep + 1;         // source values the batch spans
    const float* src = values + first;
    if (values_on_device) {
      stage.resize((size_t)count);
      if (hipMemcpyAsync(stage.data(), src, (size_t)count * sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) {
        st = marfa_set_error(MARFA_E_DEVICE, "ptbin: device-to-host copy failed");
        break;
      }
      src = stage.data();
    }
    // consecutive records are adjacent in the file; each repeats its
    // neighbour's shared end value
    rec.resize((size_t)(nb * kNT));
    for (int64_t k = 0; k < nb; ++k) std::memcpy(rec.data() + k * kNT, src + k * kStep, kNT * sizeof(float));
    if (!write_all(fd, reinterpret_cast<const char*>(rec.data()), rec.size() * sizeof(float),
                   (off_t)((r0 - 1) * kNT * (int64_t)sizeof(float)))) {
      st = io_fail("ptbin: write failed on", path);
      break;
    }
    done += nb;
  }
  if (close(fd) != 0 && st == MARFA_OK) st = io_fail("ptbin: close failed on", path);
  if (st == MARFA_OK && records_written) *records_written = (int32_t)done;
  return st;
}
