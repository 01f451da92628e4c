// marfa_io.hip -- the paper's two binary file formats, host code only:
//  * PT-table record files (Appendix A): one direct-access file per layer,
//    records of 20481 single-precision values, record r covering
//    [10 r, 10 r + 10] cm^-1 at byte offset (r - 1) * 20481 * 4;
//  * spectral line databases (Appendix B): packed 36-byte line records.
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

// ------------------------------------------------------------------
// line database (Appendix B)
// ------------------------------------------------------------------
namespace {

constexpr int64_t kRec = MARFA_LINEDB_RECORD;
static_assert(kRec == 8 + 7 * 4, "record layout");

// little-endian field codecs (the host is little-endian; memcpy keeps the
// packed record free of alignment assumptions)
template <typename T>
void put(unsigned char* p, T v) { std::memcpy(p, &v, sizeof(T)); }
template <typename T>
T get(const unsigned char* p) {
  T v;
  std::memcpy(&v, p, sizeof(T));
  return v;
}

}  // namespace

extern "C" marfa_status marfa_linedb_count(const char* path, int64_t* n) {
  if (!path || !n) return marfa_set_error(MARFA_E_INVALID, "linedb: null argument");
  *n = 0;
  const int fd = open(path, O_RDONLY);
  if (fd < 0) return io_fail("linedb: cannot open", path);
  const off_t size = lseek(fd, 0, SEEK_END);
  close(fd);
  if (size < 0) return io_fail("linedb: cannot size", path);
  if (size % kRec != 0) return marfa_set_error(MARFA_E_INVALID, "linedb: file size is not a multiple of 36 bytes");
  *n = (int64_t)(size / kRec);
  return MARFA_OK;
}

extern "C" marfa_status marfa_linedb_read(const char* path, int64_t first, int64_t count, double* nu0, float* S296,
                                          float* gamma_air, float* gamma_self, float* E_lower, float* n_air,
                                          int32_t* mol_iso, float* delta_air) {
  if (!path) return marfa_set_error(MARFA_E_INVALID, "linedb: null path");
  if (first < 0 || count < 0) return marfa_set_error(MARFA_E_INVALID, "linedb: negative range");
  if (count > 0 && (!nu0 || !S296 || !gamma_air || !gamma_self || !E_lower || !n_air || !delta_air))
    return marfa_set_error(MARFA_E_INVALID, "linedb: null array");
  int64_t n = 0;
  marfa_status st = marfa_linedb_count(path, &n);
  if (st != MARFA_OK) return st;
  if (first + count > n) return marfa_set_error(MARFA_E_INVALID, "linedb: range past the end of the file");
  const int fd = open(path, O_RDONLY);
  if (fd < 0) return io_fail("linedb: cannot open", path);
  constexpr int64_t kChunk = 1 << 16;   // records per read
  std::vector<unsigned char> buf((size_t)(std::min(count, kChunk) * kRec));
  for (int64_t done = 0; done < count && st == MARFA_OK;) {
    const int64_t k = std::min(kChunk, count - done);
    size_t want = (size_t)(k * kRec), got = 0;
    const off_t off = (off_t)((first + done) * kRec);
    while (got < want) {
      const ssize_t r = pread(fd, buf.data() + got, want - got, off + (off_t)got);
      if (r < 0 && errno == EINTR) continue;
      if (r <= 0) break;
      got += (size_t)r;
    }
    if (got != want) {
      st = io_fail("linedb: short read on", path);
      break;
    }
    for (int64_t i = 0; i < k; ++i) {
      const unsigned char* p = buf.data() + i * kRec;
      const int64_t o = done + i;
      nu0[o] = get<double>(p);
      S296[o] = get<float>(p + 8);
      gamma_air[o] = get<float>(p + 12);
      gamma_self[o] = get<float>(p + 16);
      E_lower[o] = get<float>(p + 20);
      n_air[o] = get<float>(p + 24);
      if (mol_iso) mol_iso[o] = get<int32_t>(p + 28);
      delta_air[o] = get<float>(p + 32);
    }
    done += k;
  }
  close(fd);
  return st;
}

extern "C" marfa_status marfa_linedb_write(const char* path, const marfa_lines* L) {
  if (!path || !L) return marfa_set_error(MARFA_E_INVALID, "linedb: null argument");
  if (L->n < 0) return marfa_set_error(MARFA_E_INVALID, "linedb: negative line count");
  if (L->n > 0 && (!L->nu0 || !L->S296 || !L->gamma_air || !L->gamma_self || !L->E_lower || !L->n_air ||
                   !L->delta_air))
    return marfa_set_error(MARFA_E_INVALID, "linedb: null array");
  const int fd = open(path, O_WRONLY | O_CREAT | O_TRUNC, 0644);
  if (fd < 0) return io_fail("linedb: cannot open", path);
  constexpr int64_t kChunk = 1 << 16;
  std::vector<unsigned char> buf((size_t)(std::min<int64_t>(std::max<int64_t>(L->n, 1), kChunk) * kRec));
  marfa_status st = MARFA_OK;
  for (int64_t done = 0; done < L->n;) {
    const int64_t k = std::min(kChunk, L->n - done);
    for (int64_t i = 0; i < k; ++i) {
      unsigned char* p = buf.data() + i * kRec;
      const int64_t o = done + i;
      put<double>(p, L->nu0[o]);
      put<float>(p + 8, L->S296[o]);
      put<float>(p + 12, L->gamma_air[o]);
      put<float>(p + 16, L->gamma_self[o]);
      put<float>(p + 20, L->E_lower[o]);
      put<float>(p + 24, L->n_air[o]);
      put<int32_t>(p + 28, L->mol_iso ? L->mol_iso[o] : 0);
      put<float>(p + 32, L->delta_air[o]);
    }
    if (!write_all(fd, reinterpret_cast<const char*>(buf.data()), (size_t)(k * kRec), (off_t)(done * kRec))) {
      st = io_fail("linedb: write failed on", path);
      break;
    }
    done += k;
  }
  if (close(fd) != 0 && st == MARFA_OK) st = io_fail("linedb: close failed on", path);
  return st;
}
