// Wavefront OBJ output of field lines (Sec. 4: the command line app gathers the
// lines of all particles and writes them to one joint obj file of line
// elements).  Host code only: vertex records "v x y z", then one line element
// "l a b c ..." (1-based indices) per polyline with at least two vertices.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cerrno>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/streami.h"

namespace streami {
int set_error(int code, const char* msg);  // api.hip: the thread's last-error text
int block_count(streami_field f);          // api.hip: blocks of a handle
}

namespace {

int ofail(int code, const std::string& msg) { return streami::set_error(code, msg.c_str()); }

// Buffered text output; the first failure sticks.
struct Out {
  FILE* fp = nullptr;
  std::vector<char> buf;
  bool ok = true;
  explicit Out(FILE* f) : fp(f) { buf.reserve(1 << 20); }
  void flush() {
    if (ok && !buf.empty() && std::fwrite(buf.data(), 1, buf.size(), fp) != buf.size()) ok = false;
    buf.clear();
  }
  void put(const char* s, size_t n) {
    buf.insert(buf.end(), s, s + n);
    if (buf.size() >= (1u << 20)) flush();
  }
};

}  // namespace

extern "C" {

int streami_write_obj(const char* path, int64_t n_lines, const int64_t* offsets, const float* xyz, int32_t append,
                      int64_t* vertex_base) {
  if (!path) return ofail(STREAMI_E_ARG, "path is NULL");
  if (n_lines < 0) return ofail(STREAMI_E_ARG, "n_lines must be >= 0");
  if (n_lines > 0 && (!offsets || !xyz)) return ofail(STREAMI_E_ARG, "offsets and xyz must not be NULL");
  if (n_lines > 0 && offsets[0] < 0) return ofail(STREAMI_E_ARG, "offsets[0] must be >= 0");
  for (int64_t i = 0; i < n_lines; ++i)
    if (offsets[i + 1] < offsets[i]) return ofail(STREAMI_E_ARG, "offsets must not decrease (line " + std::to_string(i) + ")");
  const int64_t base = vertex_base ? *vertex_base : 0;
  if (base < 0) return ofail(STREAMI_E_ARG, "*vertex_base must be >= 0");
  FILE* fp = std::fopen(path, append ? "ab" : "wb");
  if (!fp) return ofail(STREAMI_E_IO, std::string("cannot open ") + path + ": " + std::strerror(errno));
  Out o(fp);
  char tmp[96];
  const int64_t v0 = n_lines > 0 ? offsets[0] : 0, v1 = n_lines > 0 ? offsets[n_lines] : 0;
  for (int64_t k = v0; k < v1; ++k) {
    const int len = std::snprintf(tmp, sizeof tmp, "v %.9g %.9g %.9g\n", (double)xyz[3 * k], (double)xyz[3 * k + 1],
                                  (double)xyz[3 * k + 2]);
    o.put(tmp, (size_t)len);
  }
  for (int64_t i = 0; i < n_lines; ++i) {
    if (offsets[i + 1] - offsets[i] < 2) continue;
    o.put("l", 1);
    for (int64_t k = offsets[i]; k < offsets[i + 1]; ++k) {
      const int len = std::snprintf(tmp, sizeof tmp, " %lld", (long long)(base + (k - v0) + 1));
      o.put(tmp, (size_t)len);
    }
    o.put("\n", 1);
  }
  o.flush();
  const bool closed = std::fclose(fp) == 0;
  if (!o.ok || !closed) return ofail(STREAMI_E_IO, std::string("write to ") + path + " failed");
  if (vertex_base) *vertex_base = base + (v1 - v0);
  return STREAMI_OK;
}

int streami_write_obj_field(streami_field f, const char* path) {
  if (!f) return ofail(STREAMI_E_ARG, "field handle is NULL");
  if (!path) return ofail(STREAMI_E_ARG, "path is NULL");
  const int32_t n_blocks = streami::block_count(f);
  int rc = STREAMI_OK;
  int64_t base = 0;
  bool first = true;
  for (int32_t b = 0; b < n_blocks; ++b) {
    int64_t np = 0, nv = 0;
    if ((rc = streami_block_info(f, b, &np, &nv))) return rc;
    int64_t need = 0;
    rc = streami_fetch_lines(f, b, 0, np, nullptr, nullptr, -1, nullptr, nullptr, nullptr, &need);
    if (rc != STREAMI_OK && rc != STREAMI_E_CAPACITY) return rc;
    std::vector<int64_t> off;
    std::vector<float> xyz;
    try {
      off.resize((size_t)np + 1);
      xyz.resize((size_t)std::max<int64_t>(need, 1) * 3);
    } catch (...) {
      return ofail(STREAMI_E_NOMEM, "host buffers for block " + std::to_string(b) + " failed");
    }
    if ((rc = streami_fetch_lines(f, b, 0, np, off.data(), xyz.data(), need, nullptr, nullptr, nullptr, &need)))
      return rc;
    if ((rc = streami_write_obj(path, np, off.data(), xyz.data(), first ? 0 : 1, &base))) return rc;
    first = false;
  }
  if (first) return streami_write_obj(path, 0, nullptr, nullptr, 0, nullptr);  // no blocks: an empty file
  return STREAMI_OK;
}

}  // extern "C"
