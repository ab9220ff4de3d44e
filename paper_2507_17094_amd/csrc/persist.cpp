// Saving an index to a file and loading it back.
//
// The file holds what miann_index_import takes (per shard: the originals,
// graph, global ids, inter-shard map, ghost ids and ghost graph) plus the
// index's dimensions and types; loading imports them again, so the store,
// sign table and dense ghost arrays are rebuilt by the same kernels and the
// loaded index searches exactly like the saved one. Layout (little-endian):
//   "MIANNIX1", u32 version = 1,
//   i32 S, d, in_dtype, store_dtype, degree, ghost_degree, has_sign_table,
//   per shard: i64 n, i64 R, i32 has_next_map,
//              originals [n][d] (in_dtype, rows unpadded), graph u32[n][degree],
//              global ids u32[n], next map u32[n] (if present),
//              ghost ids u32[R], ghost graph u32[R][ghost_degree].
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <memory>
#include <vector>

#include "../../include/miann.h"

miann_status miann_fail(miann_status st, const char* fmt, ...);

namespace {

constexpr char kMagic[8] = {'M', 'I', 'A', 'N', 'N', 'I', 'X', '1'};
constexpr uint32_t kVersion = 1;

struct File {
  FILE* f = nullptr;
  ~File() {
    if (f) fclose(f);
  }
};

bool put(FILE* f, const void* p, size_t n) { return n == 0 || fwrite(p, 1, n, f) == n; }
bool get(FILE* f, void* p, size_t n) { return n == 0 || fread(p, 1, n, f) == n; }

// Device -> host copy of n bytes (synchronous).
bool d2h(void* dst, const void* src, size_t n) {
  return n == 0 || hipMemcpy(dst, src, n, hipMemcpyDeviceToHost) == hipSuccess;
}

// Device buffers freed with the loader.
struct DevBufs {
  std::vector<void*> v;
  ~DevBufs() {
    for (void* p : v) hipFree(p);
  }
  void* up(const std::vector<uint8_t>& h) {
    void* p = nullptr;
    if (hipMalloc(&p, h.empty() ? 16 : h.size()) != hipSuccess) return nullptr;
    v.push_back(p);
    if (!h.empty() && hipMemcpy(p, h.data(), h.size(), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    return p;
  }
};

}  // namespace

extern "C" {

miann_status miann_index_save(const miann_index* idx, const char* path) {
  if (!idx || !path) return miann_fail(MIANN_EINVAL, "miann_index_save: null argument");
  int32_t S = 0, d = 0, degree = 0, store_dt = 0;
  int64_t n_total = 0;
  miann_status rc = miann_index_info(idx, &S, &n_total, &d, &degree, &store_dt);
  if (rc != MIANN_OK) return rc;
  std::vector<miann_shard_view> views(S);
  for (int s = 0; s < S; s++)
    if ((rc = miann_index_shard(idx, s, &views[s])) != MIANN_OK) return rc;
  const int32_t in_dt = views[0].in_dtype, deg_g = views[0].ghost_degree;
  const int32_t has_sign = views[0].sign != nullptr;
  const size_t esize = in_dt == MIANN_U8 ? 1 : 4;
  const size_t row_bytes = (d * esize + 127) / 128 * 128;  // stored originals: rows padded to 128 bytes
  if (hipDeviceSynchronize() != hipSuccess) return miann_fail(MIANN_EDEVICE, "miann_index_save: device error");
  File fh;
  fh.f = fopen(path, "wb");
  if (!fh.f) return miann_fail(MIANN_EINVAL, "miann_index_save: cannot open %s for writing", path);
  FILE* f = fh.f;
  const int32_t hdr[7] = {S, d, in_dt, store_dt, degree, deg_g, has_sign};
  bool ok = put(f, kMagic, 8) && put(f, &kVersion, 4) && put(f, hdr, sizeof hdr);
  for (int s = 0; s < S && ok; s++) {
    const miann_shard_view& v = views[s];
    const int32_t has_next = v.next_map != nullptr;
    ok = put(f, &v.n, 8) && put(f, &v.n_ghost, 8) && put(f, &has_next, 4);
    // originals, row by row without the padding
    std::vector<uint8_t> rows((size_t)v.n * row_bytes);
    ok = ok && d2h(rows.data(), v.originals, rows.size());
    for (int64_t i = 0; i < v.n && ok; i++) ok = put(f, rows.data() + (size_t)i * row_bytes, d * esize);
    std::vector<uint8_t> buf;
    auto arr = [&](const void* src, size_t bytes) {
      buf.resize(bytes);
      return d2h(buf.data(), src, bytes) && put(f, buf.data(), bytes);
    };
    ok = ok && arr(v.graph, (size_t)v.n * degree * 4);
    if (v.global_ids) {
      ok = ok && arr(v.global_ids, (size_t)v.n * 4);
    } else {  // identity map
      std::vector<uint32_t> ident((size_t)v.n);
      for (int64_t i = 0; i < v.n; i++) ident[i] = (uint32_t)i;
      ok = ok && put(f, ident.data(), ident.size() * 4);
    }
    if (has_next) ok = ok && arr(v.next_map, (size_t)v.n * 4);
    if (v.n_ghost > 0)
      ok = ok && arr(v.ghost_ids, (size_t)v.n_ghost * 4) && arr(v.ghost_graph, (size_t)v.n_ghost * deg_g * 4);
  }
  if (!ok) return miann_fail(MIANN_EDEVICE, "miann_index_save: writing %s failed", path);
  return MIANN_OK;
}

miann_status miann_index_load(const char* path, void* stream, miann_index** out) {
  if (!path || !out) return miann_fail(MIANN_EINVAL, "miann_index_load: null argument");
  File fh;
  fh.f = fopen(path, "rb");
  if (!fh.f) return miann_fail(MIANN_EINVAL, "miann_index_load: cannot open %s", path);
  FILE* f = fh.f;
  char magic[8];
  uint32_t ver = 0;
  int32_t hdr[7];
  if (!get(f, magic, 8) || std::memcmp(magic, kMagic, 8) != 0 || !get(f, &ver, 4) || ver != kVersion ||
      !get(f, hdr, sizeof hdr))
    return miann_fail(MIANN_EINVAL, "miann_index_load: %s is not an index file of this version", path);
  const int32_t S = hdr[0], d = hdr[1], in_dt = hdr[2], store_dt = hdr[3], degree = hdr[4], deg_g = hdr[5],
                has_sign = hdr[6];
  if (S < 1 || S > 64 || d < 1 || d > 65536 || degree < 1 || degree > 1024 || deg_g < 0 || deg_g > 1024 ||
      (in_dt != MIANN_F32 && in_dt != MIANN_U8))
    return miann_fail(MIANN_EINVAL, "miann_index_load: %s has an invalid header", path);
  const size_t esize = in_dt == MIANN_U8 ? 1 : 4;
  // bytes left in the file, so that no header value can ask for more memory than the file holds
  const long pos = ftell(f);
  if (pos < 0 || fseek(f, 0, SEEK_END) != 0) return miann_fail(MIANN_EINVAL, "miann_index_load: cannot seek %s", path);
  const long end = ftell(f);
  if (end < pos || fseek(f, pos, SEEK_SET) != 0)
    return miann_fail(MIANN_EINVAL, "miann_index_load: cannot seek %s", path);
  size_t left = (size_t)(end - pos);
  DevBufs dev;
  std::vector<miann_shard_desc> desc(S);
  for (int s = 0; s < S; s++) {
    int64_t n = 0, R = 0;
    int32_t has_next = 0;
    if (left < 20 || !get(f, &n, 8) || !get(f, &R, 8) || !get(f, &has_next, 4) || n < 1 || R < 0 || R > n ||
        (uint64_t)n > (uint64_t)left)
      return miann_fail(MIANN_EINVAL, "miann_index_load: %s: bad shard %d header", path, s);
    left -= 20;
    // the shard's arrays must all be in the file before anything is allocated on the device
    const uint64_t need = (uint64_t)n * ((uint64_t)d * esize + (uint64_t)degree * 4 + 4 + (has_next ? 4 : 0)) +
                          (uint64_t)R * (4 + (uint64_t)deg_g * 4);
    if (need > (uint64_t)left)
      return miann_fail(MIANN_EINVAL, "miann_index_load: %s is truncated (shard %d)", path, s);
    left -= (size_t)need;
    auto read_up = [&](size_t bytes, const void** dst) {
      std::vector<uint8_t> h(bytes);
      if (!get(f, h.data(), bytes)) return false;
      *dst = dev.up(h);
      return *dst != nullptr;
    };
    miann_shard_desc& sd = desc[s];
    std::memset(&sd, 0, sizeof sd);
    sd.n = n;
    sd.n_ghost = R;
    const void* p = nullptr;
    bool ok = read_up((size_t)n * d * esize, &p);
    sd.vectors = p;
    ok = ok && read_up((size_t)n * degree * 4, &p);
    sd.graph = (const uint32_t*)p;
    ok = ok && read_up((size_t)n * 4, &p);
    sd.global_ids = (const uint32_t*)p;
    if (ok && has_next) {
      ok = read_up((size_t)n * 4, &p);
      sd.next_map = (const uint32_t*)p;
    }
    if (ok && R > 0) {
      ok = read_up((size_t)R * 4, &p);
      sd.ghost_ids = (const uint32_t*)p;
      ok = ok && read_up((size_t)R * deg_g * 4, &p);
      sd.ghost_graph = (const uint32_t*)p;
    }
    if (!ok) return miann_fail(MIANN_EDEVICE, "miann_index_load: reading %s or copying it to the device failed", path);
  }
  const miann_status rc = miann_index_import(desc.data(), S, d, in_dt, store_dt, degree, deg_g, has_sign, stream, out);
  // nothing queued may still read the staging buffers when they are freed on return
  hipStreamSynchronize((hipStream_t)stream);
  return rc;
}

}  // extern "C"
