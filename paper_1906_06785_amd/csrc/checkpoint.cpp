// Checkpoint files of a TT pair (the Picard iterate of Alg. 3.1 is the
// natural restart point) and parameter files of the learned correction's
// network: host-side formats, written and read with stdio.
//
// Layout, little-endian:
//   8 bytes  "SGTTPAIR"
//   uint32   format version (1)
//   uint32   number of TTs (2: velocity, pressure)
//   per TT:  int32 n1, n2, n3, r1, r2
//   per TT:  core 1 (n1 x r1, row-major), core 2 (r1 x n2 x r2), core 3
//            (n3 x r2, row-major), as IEEE float64
//   uint64   FNV-1a hash of every byte above
#include "checkpoint.h"

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "sgtt.h"

namespace sgtt {
namespace {

constexpr char kMagic[8] = {'S', 'G', 'T', 'T', 'P', 'A', 'I', 'R'};
constexpr uint32_t kVersion = 1;
constexpr long kMaxDim = 1L << 31;

struct Fnv {
  uint64_t h = 1469598103934665603ull;
  void add(const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
      h ^= b[i];
      h *= 1099511628211ull;
    }
  }
};

struct FileCloser {
  void operator()(FILE* f) const {
    if (f) std::fclose(f);
  }
};
using File = std::unique_ptr<FILE, FileCloser>;

bool write_all(FILE* f, Fnv& h, const void* p, size_t n) {
  h.add(p, n);
  return std::fwrite(p, 1, n, f) == n;
}
bool read_all(FILE* f, Fnv& h, void* p, size_t n) {
  if (std::fread(p, 1, n, f) != n) return false;
  h.add(p, n);
  return true;
}

bool dims_valid(const int* d) {
  for (int q = 0; q < 2; ++q) {
    const int* e = d + 5 * q;
    for (int i = 0; i < 5; ++i)
      if (e[i] < 1) return false;
    // a TT's ranks never exceed what its cores can hold
    if ((long)e[0] * e[3] >= kMaxDim || (long)e[3] * e[1] * e[4] >= kMaxDim || (long)e[2] * e[4] >= kMaxDim)
      return false;
  }
  return true;
}

long core_len(const int* e, int which) {
  return which == 0 ? (long)e[0] * e[3] : which == 1 ? (long)e[3] * e[1] * e[4] : (long)e[2] * e[4];
}

// header and dims; returns 0 or an error status
int read_header(FILE* f, Fnv& h, int* dims) {
  char magic[8];
  uint32_t ver = 0, ntt = 0;
  if (!read_all(f, h, magic, 8) || std::memcmp(magic, kMagic, 8) != 0) return SGTT_E_IO;
  if (!read_all(f, h, &ver, 4) || ver != kVersion) return SGTT_E_IO;
  if (!read_all(f, h, &ntt, 4) || ntt != 2) return SGTT_E_IO;
  int32_t d[10];
  if (!read_all(f, h, d, sizeof(d))) return SGTT_E_IO;
  for (int i = 0; i < 10; ++i) dims[i] = d[i];
  if (!dims_valid(dims)) return SGTT_E_IO;
  return SGTT_OK;
}

}  // namespace

int pair_file_write(const char* path, const int* dims, const double* const* cores) {
  if (!path || !dims || !cores || !dims_valid(dims)) return SGTT_E_INVALID;
  for (int i = 0; i < 6; ++i)
    if (!cores[i]) return SGTT_E_INVALID;
  // write to a temporary name and rename, so a crash never leaves a torn file
  const std::string tmp = std::string(path) + ".tmp";
  {
    File f(std::fopen(tmp.c_str(), "wb"));
    if (!f) return SGTT_E_IO;
    Fnv h;
    const uint32_t ver = kVersion, ntt = 2;
    int32_t d[10];
    for (int i = 0; i < 10; ++i) d[i] = dims[i];
    bool ok = write_all(f.get(), h, kMagic, 8) && write_all(f.get(), h, &ver, 4) && write_all(f.get(), h, &ntt, 4) &&
              write_all(f.get(), h, d, sizeof(d));
    for (int q = 0; ok && q < 2; ++q)
      for (int w = 0; ok && w < 3; ++w)
        ok = write_all(f.get(), h, cores[3 * q + w], sizeof(double) * (size_t)core_len(dims + 5 * q, w));
    const uint64_t sum = h.h;
    ok = ok && std::fwrite(&sum, 1, 8, f.get()) == 8;
    ok = ok && std::fflush(f.get()) == 0;
    if (!ok) {
      f.reset();
      std::remove(tmp.c_str());
      return SGTT_E_IO;
    }
  }
  if (std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return SGTT_E_IO;
  }
  return SGTT_OK;
}

int pair_file_info(const char* path, int* dims) {
  if (!path || !dims) return SGTT_E_INVALID;
  File f(std::fopen(path, "rb"));
  if (!f) return SGTT_E_IO;
  Fnv h;
  return read_header(f.get(), h, dims);
}

int pair_file_read(const char* path, const int* caps, double* const* cores, int* dims) {
  if (!path || !caps || !cores || !dims) return SGTT_E_INVALID;
  for (int i = 0; i < 6; ++i)
    if (!cores[i]) return SGTT_E_INVALID;
  File f(std::fopen(path, "rb"));
  if (!f) return SGTT_E_IO;
  Fnv h;
  int d[10];
  int st = read_header(f.get(), h, d);
  if (st != SGTT_OK) return st;
  // caps: per TT n1, n2, n3, cap1, cap2 of the caller's buffers
  for (int q = 0; q < 2; ++q) {
    const int* e = d + 5 * q;
    const int* c = caps + 5 * q;
    if (e[0] != c[0] || e[1] != c[1] || e[2] != c[2]) return SGTT_E_INVALID;
    if (e[3] > c[3] || e[4] > c[4]) return SGTT_E_RANK_CAP;
  }
  // read into staging first: the caller's buffers change only when the
  // whole file has been read and its hash checked
  std::vector<double> stage[6];
  for (int q = 0; q < 2; ++q)
    for (int w = 0; w < 3; ++w) {
      std::vector<double>& v = stage[3 * q + w];
      v.resize((size_t)core_len(d + 5 * q, w));
      if (!read_all(f.get(), h, v.data(), sizeof(double) * v.size())) return SGTT_E_IO;
    }
  uint64_t sum = 0;
  if (std::fread(&sum, 1, 8, f.get()) != 8 || sum != h.h) return SGTT_E_IO;
  for (int i = 0; i < 6; ++i) std::memcpy(cores[i], stage[i].data(), sizeof(double) * stage[i].size());
  for (int i = 0; i < 10; ++i) dims[i] = d[i];
  return SGTT_OK;
}

// ---------------------------------------------------------------- networks
// Parameter files of the learned correction's network, little-endian:
//   8 bytes  "SGTTMLPN"
//   uint32   format version (1)
//   int32    n (input and output length), width (hidden layer width)
//   int64    nparam = w n + w + w w + w + n w + n
//   nparam   IEEE float32 parameters [W1, b1, W2, b2, W3, b3], row-major
//   uint64   FNV-1a hash of every byte above
namespace {
constexpr char kNetMagic[8] = {'S', 'G', 'T', 'T', 'M', 'L', 'P', 'N'};

long net_params(long n, long w) { return w * n + w + w * w + w + n * w + n; }

bool net_dims_valid(long n, long w, long np) {
  return n >= 1 && w >= 1 && n < kMaxDim && w < kMaxDim && np == net_params(n, w) && np < (1L << 40);
}

int read_net_header(FILE* f, Fnv& h, int* n, int* w, long* np) {
  char magic[8];
  uint32_t ver = 0;
  int32_t d[2];
  int64_t p = 0;
  if (!read_all(f, h, magic, 8) || std::memcmp(magic, kNetMagic, 8) != 0) return SGTT_E_IO;
  if (!read_all(f, h, &ver, 4) || ver != kVersion) return SGTT_E_IO;
  if (!read_all(f, h, d, sizeof(d)) || !read_all(f, h, &p, 8)) return SGTT_E_IO;
  if (!net_dims_valid(d[0], d[1], (long)p)) return SGTT_E_IO;
  *n = d[0];
  *w = d[1];
  *np = (long)p;
  return SGTT_OK;
}
}  // namespace

int net_file_write(const char* path, int n, int w, long nparam, const float* params) {
  if (!path || !params || !net_dims_valid(n, w, nparam)) return SGTT_E_INVALID;
  const std::string tmp = std::string(path) + ".tmp";
  {
    File f(std::fopen(tmp.c_str(), "wb"));
    if (!f) return SGTT_E_IO;
    Fnv h;
    const uint32_t ver = kVersion;
    const int32_t d[2] = {n, w};
    const int64_t p = nparam;
    bool ok = write_all(f.get(), h, kNetMagic, 8) && write_all(f.get(), h, &ver, 4) &&
              write_all(f.get(), h, d, sizeof(d)) && write_all(f.get(), h, &p, 8) &&
              write_all(f.get(), h, params, sizeof(float) * (size_t)nparam);
    const uint64_t sum = h.h;
    ok = ok && std::fwrite(&sum, 1, 8, f.get()) == 8;
    ok = ok && std::fflush(f.get()) == 0;
    if (!ok) {
      f.reset();
      std::remove(tmp.c_str());
      return SGTT_E_IO;
    }
  }
  if (std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return SGTT_E_IO;
  }
  return SGTT_OK;
}

int net_file_info(const char* path, int* n, int* w, long* nparam) {
  if (!path || !n || !w || !nparam) return SGTT_E_INVALID;
  File f(std::fopen(path, "rb"));
  if (!f) return SGTT_E_IO;
  Fnv h;
  return read_net_header(f.get(), h, n, w, nparam);
}

int net_file_read(const char* path, int n, int w, float* params) {
  if (!path || !params || n < 1 || w < 1) return SGTT_E_INVALID;
  File f(std::fopen(path, "rb"));
  if (!f) return SGTT_E_IO;
  Fnv h;
  int fn = 0, fw = 0;
  long np = 0;
  const int st = read_net_header(f.get(), h, &fn, &fw, &np);
  if (st != SGTT_OK) return st;
  if (fn != n || fw != w) return SGTT_E_INVALID;   // a network of another shape
  // staging first: the caller's parameters change only after the hash check
  std::vector<float> stage((size_t)np);
  if (!read_all(f.get(), h, stage.data(), sizeof(float) * stage.size())) return SGTT_E_IO;
  uint64_t sum = 0;
  if (std::fread(&sum, 1, 8, f.get()) != 8 || sum != h.h) return SGTT_E_IO;
  std::memcpy(params, stage.data(), sizeof(float) * stage.size());
  return SGTT_OK;
}

}  // namespace sgtt

extern "C" {

int sgtt_mlp_file_write_host(const char* path, int n, int width, const float* params) {
  return sgtt::net_file_write(path, n, width, sgtt::net_params(n, width), params);
}

int sgtt_mlp_file_info(const char* path, int* n, int* width, long* nparam) {
  return sgtt::net_file_info(path, n, width, nparam);
}

int sgtt_mlp_file_read_host(const char* path, int n, int width, float* params) {
  return sgtt::net_file_read(path, n, width, params);
}

int sgtt_pair_file_write_host(const char* path, const int* dims, const double* const* cores) {
  return sgtt::pair_file_write(path, dims, cores);
}

int sgtt_pair_file_info(const char* path, int* dims) { return sgtt::pair_file_info(path, dims); }

int sgtt_pair_file_read_host(const char* path, const int* caps, double* const* cores, int* dims) {
  return sgtt::pair_file_read(path, caps, cores, dims);
}

}  // extern "C"
