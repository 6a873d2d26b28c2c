// Index file: reader, writer and validation of the tables.
//
// Layout (little-endian): a 256-byte header, then these sections, each starting
// at a 64-byte-aligned offset: attr_sorted i64[n], ext_id i64[n],
// seg_start i64[S+1], seg_entry i32[S], seg_maxlevel i32[S], level u8[n],
// uprow i32[n], vectors f32[n*d], adj0 i32[n*S*M0], gbits0 u32[n*W0],
// adjU i32[R*S*MU], gbitsU u32[R*WU]; then padding to 64 bytes and a CRC-32
// (IEEE 802.3, reflected) of every preceding byte.
//
// The tables hold the index of Sec. 4.1: per node and layer, S chunks of at
// most M ids (-1 padded, chunk j holding neighbours in segment j) and a bitmap
// of ceil(S M / 32) words marking the global (post-filter) edges; bit
// j * M + r marks entry r of chunk j.  The skip-list successor is implicit:
// internal ids are ranks in attribute order.
#include <algorithm>
#include <atomic>
#include <thread>
#include <vector>
#include <cstdio>
#include <cstring>

#include "unify_internal.h"

namespace unify {
namespace {

constexpr char kMagic[8] = {'U', 'N', 'I', 'F', 'Y', 'I', 'X', '1'};
constexpr uint32_t kVersion = 1;

#pragma pack(push, 1)
struct FileHeader {
  char magic[8];
  uint32_t version;
  uint32_t flags;
  int64_t n;
  int32_t d, S, M0, MU, L, ef_cons, gentry, reserved;
  double mL;
  uint64_t seed;
  int64_t R;
  int32_t W0, WU;
  uint8_t zero[168];
};
#pragma pack(pop)
static_assert(sizeof(FileHeader) == 256, "index file header is 256 bytes");

// Bitwise CRC-32 (polynomial 0x04C11DB7 reflected), byte at a time via a
// 16-entry nibble table.
uint32_t crc_nibble(uint32_t crc, const uint8_t* p, size_t n) {
  static const uint32_t T[16] = {
      0x00000000u, 0x1DB71064u, 0x3B6E20C8u, 0x26D930ACu, 0x76DC4190u, 0x6B6B51F4u,
      0x4DB26158u, 0x5005713Cu, 0xEDB88320u, 0xF00F9344u, 0xD6D6A3E8u, 0xCB61B38Cu,
      0x9B64C2B0u, 0x86D3D2D4u, 0xA00AE278u, 0xBDBDF21Cu};
  for (size_t i = 0; i < n; ++i) {
    crc ^= p[i];
    crc = (crc >> 4) ^ T[crc & 15u];
    crc = (crc >> 4) ^ T[crc & 15u];
  }
  return crc;
}

struct Sink {
  FILE* f = nullptr;
  uint64_t pos = 0;
  uint32_t crc = 0xFFFFFFFFu;
  bool ok = true;
  void write(const void* p, size_t n) {
    if (!n) return;
    ok = ok && std::fwrite(p, 1, n, f) == n;
    crc = crc_nibble(crc, static_cast<const uint8_t*>(p), n);
    pos += n;
  }
  void pad64() {
    static const uint8_t zeros[64] = {};
    write(zeros, (64 - pos % 64) % 64);
  }
};

struct Source {
  const uint8_t* base;
  size_t size;
  size_t pos = 0;
  bool ok = true;
  template <class T>
  void section(std::vector<T>& out, size_t count) {
    pos = (pos + 63) & ~size_t(63);
    if (count > (size - pos) / sizeof(T)) {
      ok = false;
      return;
    }
    out.resize(count);
    if (count) std::memcpy(out.data(), base + pos, count * sizeof(T));
    pos += count * sizeof(T);
  }
};

}  // namespace

int read_index_file(const char* path, HostIndex& H, std::string& err) {
  FILE* f = std::fopen(path, "rb");
  if (!f) {
    err = std::string("cannot open index file ") + path;
    return UNIFY_EIO;
  }
  std::fseek(f, 0, SEEK_END);
  long long sz = std::ftell(f);
  std::fseek(f, 0, SEEK_SET);
  if (sz < (long long)sizeof(FileHeader) + 4) {
    std::fclose(f);
    err = "index file too short";
    return UNIFY_EFORMAT;
  }
  std::vector<uint8_t> buf((size_t)sz);
  size_t got = std::fread(buf.data(), 1, buf.size(), f);
  std::fclose(f);
  if (got != buf.size()) {
    err = "short read of index file";
    return UNIFY_EIO;
  }
  FileHeader h;
  std::memcpy(&h, buf.data(), sizeof h);
  if (std::memcmp(h.magic, kMagic, 8) != 0) {
    err = "not an index file (bad magic)";
    return UNIFY_EFORMAT;
  }
  if (h.version != kVersion) {
    err = "unsupported index file version";
    return UNIFY_EFORMAT;
  }
  uint32_t stored;
  std::memcpy(&stored, buf.data() + buf.size() - 4, 4);
  uint32_t crc = crc_nibble(0xFFFFFFFFu, buf.data(), buf.size() - 4) ^ 0xFFFFFFFFu;
  if (crc != stored) {
    err = "index file checksum mismatch";
    return UNIFY_EFORMAT;
  }
  if (h.n < 1 || h.n >= (int64_t(1) << 31) || h.d < 4 || h.d % 4 || h.d > 4096 || h.S < 1 ||
      h.S > 64 || h.M0 < 1 || h.M0 > 128 || h.MU < 1 || h.MU > 128 || h.R < 0 || h.L < 0 ||
      h.L > 30 || h.W0 != (h.S * h.M0 + 31) / 32 || h.WU != (h.S * h.MU + 31) / 32) {
    err = "index file header out of range";
    return UNIFY_EFORMAT;
  }
  H.n = h.n;
  H.d = h.d;
  H.S = h.S;
  H.M0 = h.M0;
  H.MU = h.MU;
  H.L = h.L;
  H.ef_cons = h.ef_cons;
  H.gentry = h.gentry;
  H.mL = h.mL;
  H.seed = h.seed;
  H.R = h.R;
  H.W0 = h.W0;
  H.WU = h.WU;
  Source src{buf.data(), buf.size() - 4, sizeof(FileHeader)};
  const size_t n = (size_t)h.n, S = (size_t)h.S, R = (size_t)h.R;
  src.section(H.attr, n);
  src.section(H.ext, n);
  src.section(H.seg_start, S + 1);
  src.section(H.seg_entry, S);
  src.section(H.seg_maxlevel, S);
  src.section(H.level, n);
  src.section(H.uprow, n);
  src.section(H.vec, n * (size_t)h.d);
  src.section(H.adj0, n * S * (size_t)h.M0);
  src.section(H.gbits0, n * (size_t)h.W0);
  src.section(H.adjU, R * S * (size_t)h.MU);
  src.section(H.gbitsU, R * (size_t)h.WU);
  if (!src.ok || ((src.pos + 63) & ~size_t(63)) != src.size) {
    err = "index file sections do not match the header";
    return UNIFY_EFORMAT;
  }
  return validate_index(H, err);
}

int validate_index(const HostIndex& H, std::string& err) {
  const int64_t n = H.n;
  for (int64_t i = 1; i < n; ++i)
    if (H.attr[i] < H.attr[i - 1]) {
      err = "attributes are not sorted";
      return UNIFY_EFORMAT;
    }
  if (H.seg_start[0] != 0 || H.seg_start[H.S] != n) {
    err = "segment table does not cover the objects";
    return UNIFY_EFORMAT;
  }
  for (int j = 0; j < H.S; ++j) {
    if (H.seg_start[j + 1] < H.seg_start[j]) {
      err = "segment table is not monotone";
      return UNIFY_EFORMAT;
    }
    int32_t e = H.seg_entry[j];
    bool empty = H.seg_start[j + 1] == H.seg_start[j];
    if (empty ? (e != -1) : (e < H.seg_start[j] || e >= H.seg_start[j + 1] ||
                             H.level[e] != H.seg_maxlevel[j])) {
      err = "bad segment entry";
      return UNIFY_EFORMAT;
    }
  }
  if (H.gentry < 0 || H.gentry >= n || H.level[H.gentry] != H.L) {
    err = "bad global entry";
    return UNIFY_EFORMAT;
  }
  int64_t rows = 0;
  for (int64_t v = 0; v < n; ++v) {
    if (H.level[v] > H.L) {
      err = "node level above the top level";
      return UNIFY_EFORMAT;
    }
    if (H.level[v] == 0 ? H.uprow[v] != -1 : H.uprow[v] != rows) {
      err = "upper-row table is inconsistent";
      return UNIFY_EFORMAT;
    }
    rows += H.level[v];
  }
  if (rows != H.R) {
    err = "upper-row count mismatch";
    return UNIFY_EFORMAT;
  }
  // every edge names an object that exists on that layer (object ranges checked in parallel)
  const int nt = (int)std::max<int64_t>(1, std::min<int64_t>({16, (int64_t)std::thread::hardware_concurrency(),
                                                                n / 65536 + 1}));
  std::atomic<bool> bad{false};
  auto check = [&](int64_t v0, int64_t v1) {
    for (int64_t v = v0; v < v1 && !bad.load(std::memory_order_relaxed); ++v) {
      for (int l = 0; l <= H.level[v]; ++l) {
        const int mc = l == 0 ? H.M0 : H.MU;
        const int32_t* row = l == 0 ? &H.adj0[(size_t)v * H.S * mc]
                                    : &H.adjU[(size_t)(H.uprow[v] + l - 1) * H.S * mc];
        for (int t = 0; t < H.S * mc; ++t) {
          int32_t x = row[t];
          if (x == -1) continue;
          if (x < 0 || x >= n || H.level[x] < l) bad = true;
        }
      }
    }
  };
  std::vector<std::thread> pool;
  for (int i = 0; i < nt; ++i) pool.emplace_back(check, n * i / nt, n * (i + 1) / nt);
  for (auto& t : pool) t.join();
  if (bad) {
    err = "adjacency entry out of range";
    return UNIFY_EFORMAT;
  }
  return UNIFY_OK;
}

int write_index_file(const char* path, const HostIndex& H, std::string& err) {
  FILE* f = std::fopen(path, "wb");
  if (!f) {
    err = std::string("cannot create ") + path;
    return UNIFY_EIO;
  }
  Sink s;
  s.f = f;
  FileHeader h;
  std::memset(&h, 0, sizeof h);
  std::memcpy(h.magic, kMagic, 8);
  h.version = kVersion;
  h.n = H.n;
  h.d = H.d;
  h.S = H.S;
  h.M0 = H.M0;
  h.MU = H.MU;
  h.L = H.L;
  h.ef_cons = H.ef_cons;
  h.gentry = H.gentry;
  h.mL = H.mL;
  h.seed = H.seed;
  h.R = H.R;
  h.W0 = H.W0;
  h.WU = H.WU;
  s.write(&h, sizeof h);
  auto sec = [&](const auto& v) {
    s.pad64();
    s.write(v.data(), v.size() * sizeof(v[0]));
  };
  sec(H.attr);
  sec(H.ext);
  sec(H.seg_start);
  sec(H.seg_entry);
  sec(H.seg_maxlevel);
  sec(H.level);
  sec(H.uprow);
  sec(H.vec);
  sec(H.adj0);
  sec(H.gbits0);
  sec(H.adjU);
  sec(H.gbitsU);
  s.pad64();
  uint32_t crc = s.crc ^ 0xFFFFFFFFu;
  bool ok = s.ok && std::fwrite(&crc, 4, 1, f) == 1;
  ok = std::fclose(f) == 0 && ok;
  if (!ok) {
    err = std::string("write failed: ") + path;
    return UNIFY_EIO;
  }
  return UNIFY_OK;
}

}  // namespace unify
