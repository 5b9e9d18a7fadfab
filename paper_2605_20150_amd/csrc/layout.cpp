// Layout build (Sec. 3.3): Morton order of the Gaussian centres, so that
// contiguous runs of B rows (the blocks) are spatially compact.  In memory
// (tide_morton_order) or out of core (tide_layout_build: sorted runs on
// disk, then a k-way merge that streams the blocks into the base segment).
#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <queue>
#include <string>
#include <thread>
#include <vector>

#include "common.h"

using namespace tide;

namespace {

constexpr double kCells = 2097152.0;   // 2^21 per axis

// Spreads the low 21 bits of v so that bit i lands on bit 3 i.
inline uint64_t spread3(uint64_t v) {
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x1f00000000ffffull;
  v = (v | (v << 16)) & 0x1f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

// The quantisation both layout paths use: cell = floor((x - lo) * scale),
// clamped to [0, 2^21 - 1], scale = 2^21 / (hi - lo) (0 on a flat axis).
struct MortonGrid {
  double lo[3], scale[3];
  void set(const double* lo_, const double* hi_) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = lo_[a];
      scale[a] = hi_[a] > lo_[a] ? kCells / (hi_[a] - lo_[a]) : 0.0;
    }
  }
  uint64_t code(const float* xyz) const {
    uint64_t c = 0;
    for (int a = 0; a < 3; ++a) {
      const double q = std::floor((xyz[a] - lo[a]) * scale[a]);
      const uint64_t u = (uint64_t)std::min(kCells - 1.0, std::max(0.0, q));
      c |= spread3(u) << a;
    }
    return c;
  }
};

}  // namespace

extern "C" tide_status tide_morton_order(const float* xyz, int64_t n, int64_t stride, int64_t* perm) {
  TIDE_CHECK_ARG(n >= 0 && stride >= 3, "need n >= 0 and stride >= 3");
  if (n == 0) return TIDE_OK;
  TIDE_CHECK_ARG(xyz && perm, "null argument");
  double lo[3], hi[3];
  for (int a = 0; a < 3; ++a) lo[a] = hi[a] = xyz[a];
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      const double v = xyz[i * stride + a];
      TIDE_CHECK_ARG(std::isfinite(v), "non-finite centre at row %lld", (long long)i);
      lo[a] = std::min(lo[a], v);
      hi[a] = std::max(hi[a], v);
    }
  MortonGrid grid;
  grid.set(lo, hi);
  // (code, row) pairs are unique, so an unstable sort of the pairs is the
  // stable order by code; chunks are sorted on threads and merged pairwise.
  std::vector<std::pair<uint64_t, int64_t>> kv((size_t)n);
  auto fill = [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) kv[(size_t)i] = {grid.code(xyz + i * stride), i};
  };
  const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(16, n / 65536));
  std::vector<int64_t> cut(nt + 1);
  for (int k = 0; k <= nt; ++k) cut[k] = n * k / nt;
  {
    std::vector<std::thread> th;
    for (int k = 0; k < nt; ++k)
      th.emplace_back([&, k] {
        fill(cut[k], cut[k + 1]);
        std::sort(kv.begin() + cut[k], kv.begin() + cut[k + 1]);
      });
    for (auto& t : th) t.join();
  }
  for (int width = 1; width < nt; width *= 2) {
    std::vector<std::thread> th;
    for (int k = 0; k + width < nt; k += 2 * width) {
      const int64_t a = cut[k], m = cut[k + width], b = cut[std::min(nt, k + 2 * width)];
      th.emplace_back([&, a, m, b] { std::inplace_merge(kv.begin() + a, kv.begin() + m, kv.begin() + b); });
    }
    for (auto& t : th) t.join();
  }
  for (int64_t i = 0; i < n; ++i) perm[i] = kv[(size_t)i].second;
  return TIDE_OK;
}

// ------------------------------------------------------------------------
// Out-of-core layout build.  Pass 1 reads the table once for the bounding
// box of the centres; pass 2 cuts it into runs of run_rows rows, sorts each
// run by (code, row) and writes it to tmp_dir as records (code, row, 59
// floats); pass 3 merges the runs with a heap and hands every B rows to
// tide_store_put_block.  The order equals tide_morton_order's.
namespace {

constexpr int kCols59 = 59;
constexpr size_t kRowBytes = kCols59 * sizeof(float);
constexpr size_t kRecBytes = 16 + kRowBytes;   // code u64, row i64, params

struct Fd {
  int fd = -1;
  ~Fd() {
    if (fd >= 0) ::close(fd);
  }
};

tide_status io_fail(const char* what, const std::string& path) {
  set_error("%s %s (%s)", what, path.c_str(), std::strerror(errno));
  return TIDE_EIO;
}

bool read_full(int fd, void* dst, size_t n, off_t off) {
  size_t got = 0;
  while (got < n) {
    const ssize_t r = ::pread(fd, (char*)dst + got, n - got, off + (off_t)got);
    if (r <= 0) return false;
    got += (size_t)r;
  }
  return true;
}

bool write_full(int fd, const void* src, size_t n) {
  size_t put = 0;
  while (put < n) {
    const ssize_t r = ::write(fd, (const char*)src + put, n - put);
    if (r <= 0) return false;
    put += (size_t)r;
  }
  return true;
}

// Buffered sequential reader of one run file.
struct RunReader {
  int fd = -1;
  int64_t left = 0;        // records not yet handed out
  off_t off = 0;
  std::vector<char> buf;
  size_t pos = 0, have = 0;
  bool next(const char** rec) {
    if (pos == have) {
      if (left == 0) return false;
      const size_t want = std::min<size_t>(buf.size() / kRecBytes, (size_t)left) * kRecBytes;
      if (!read_full(fd, buf.data(), want, off)) return false;
      off += (off_t)want;
      have = want;
      pos = 0;
    }
    *rec = buf.data() + pos;
    pos += kRecBytes;
    --left;
    return true;
  }
};

}  // namespace

extern "C" tide_status tide_layout_build(tide_residency* res, const char* table_path, const char* tmp_dir,
                                         int64_t run_rows) {
  TIDE_CHECK_ARG(res && table_path && tmp_dir, "null argument");
  int64_t n_rows = 0;
  int32_t block_rows = 0;
  residency_shape(res, &n_rows, &block_rows);
  TIDE_CHECK_ARG(n_rows >= 1 && run_rows >= 1, "bad sizes");
  const int64_t n_runs = (n_rows + run_rows - 1) / run_rows;
  TIDE_CHECK_ARG(n_runs <= 512, "%lld runs: raise run_rows (at most 512 runs, one open file each)",
                 (long long)n_runs);
  Fd in;
  in.fd = ::open(table_path, O_RDONLY);
  if (in.fd < 0) return io_fail("cannot open", table_path);
  {
    struct stat stt;
    if (::fstat(in.fd, &stt) != 0) return io_fail("cannot stat", table_path);
    TIDE_CHECK_ARG((int64_t)stt.st_size == n_rows * (int64_t)kRowBytes,
                   "table %s holds %lld bytes, expected %lld rows of 59 f32", table_path,
                   (long long)stt.st_size, (long long)n_rows);
  }
  // pass 1: bounding box of the centres
  const int64_t chunk = std::min<int64_t>(run_rows, n_rows);
  std::vector<float> rows((size_t)chunk * kCols59);
  double lo[3], hi[3];
  for (int64_t r0 = 0; r0 < n_rows; r0 += chunk) {
    const int64_t m = std::min(chunk, n_rows - r0);
    if (!read_full(in.fd, rows.data(), (size_t)m * kRowBytes, (off_t)(r0 * (int64_t)kRowBytes)))
      return io_fail("short read of", table_path);
    for (int64_t i = 0; i < m; ++i)
      for (int a = 0; a < 3; ++a) {
        const double v = rows[(size_t)i * kCols59 + a];
        TIDE_CHECK_ARG(std::isfinite(v), "non-finite centre at row %lld", (long long)(r0 + i));
        if (r0 == 0 && i == 0) lo[a] = hi[a] = v;
        lo[a] = std::min(lo[a], v);
        hi[a] = std::max(hi[a], v);
      }
  }
  MortonGrid grid;
  grid.set(lo, hi);
  // pass 2: sorted runs
  std::vector<std::string> names;
  auto cleanup = [&] {
    for (const auto& nm : names) ::unlink(nm.c_str());
  };
  std::vector<char> out;
  for (int64_t r0 = 0, run = 0; r0 < n_rows; r0 += chunk, ++run) {
    const int64_t m = std::min(chunk, n_rows - r0);
    if (!read_full(in.fd, rows.data(), (size_t)m * kRowBytes, (off_t)(r0 * (int64_t)kRowBytes))) {
      cleanup();
      return io_fail("short read of", table_path);
    }
    std::vector<std::pair<uint64_t, int64_t>> kv((size_t)m);
    for (int64_t i = 0; i < m; ++i) kv[(size_t)i] = {grid.code(&rows[(size_t)i * kCols59]), r0 + i};
    std::sort(kv.begin(), kv.end());
    out.resize((size_t)m * kRecBytes);
    for (int64_t i = 0; i < m; ++i) {
      char* o = out.data() + (size_t)i * kRecBytes;
      std::memcpy(o, &kv[(size_t)i].first, 8);
      std::memcpy(o + 8, &kv[(size_t)i].second, 8);
      std::memcpy(o + 16, &rows[(size_t)(kv[(size_t)i].second - r0) * kCols59], kRowBytes);
    }
    char nm[64];
    std::snprintf(nm, sizeof(nm), "/tide_run_%05lld.bin", (long long)run);
    names.push_back(std::string(tmp_dir) + nm);
    Fd f;
    f.fd = ::open(names.back().c_str(), O_WRONLY | O_CREAT | O_TRUNC, 0600);
    if (f.fd < 0 || !write_full(f.fd, out.data(), out.size())) {
      const tide_status st = io_fail("cannot write the run", names.back());
      cleanup();
      return st;
    }
  }
  std::vector<float>().swap(rows);
  std::vector<char>().swap(out);
  // pass 3: k-way merge into blocks
  std::vector<RunReader> rd(names.size());
  std::vector<Fd> fds(names.size());
  const size_t rbuf = std::max<size_t>(kRecBytes, ((size_t)4 << 20) / kRecBytes * kRecBytes);
  for (size_t r = 0; r < names.size(); ++r) {
    fds[r].fd = ::open(names[r].c_str(), O_RDONLY);
    if (fds[r].fd < 0) {
      const tide_status st = io_fail("cannot reopen the run", names[r]);
      cleanup();
      return st;
    }
    rd[r].fd = fds[r].fd;
    rd[r].left = std::min(chunk, n_rows - (int64_t)r * chunk);
    rd[r].buf.resize(rbuf);
  }
  using Item = std::pair<std::pair<uint64_t, int64_t>, int32_t>;   // ((code, row), run)
  std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
  std::vector<const char*> cur(names.size(), nullptr);
  auto push = [&](int32_t r) -> bool {
    if (!rd[r].next(&cur[r])) return rd[r].left == 0;
    uint64_t c;
    int64_t row;
    std::memcpy(&c, cur[r], 8);
    std::memcpy(&row, cur[r] + 8, 8);
    heap.push({{c, row}, r});
    return true;
  };
  for (int32_t r = 0; r < (int32_t)names.size(); ++r)
    if (!push(r)) {
      cleanup();
      return io_fail("short read of the run", names[r]);
    }
  std::vector<float> rm((size_t)block_rows * kCols59);    // the block's rows, row-major
  std::vector<float> blk((size_t)block_rows * kCols59);   // [59][rows of the block]
  int64_t done = 0, block = 0;
  while (done < n_rows) {
    const int64_t rows_k = std::min<int64_t>(block_rows, n_rows - block * (int64_t)block_rows);
    for (int64_t i = 0; i < rows_k; ++i) {
      if (heap.empty()) {
        cleanup();
        set_error("layout merge ran dry at row %lld", (long long)done);
        return TIDE_EIO;
      }
      const int32_t r = heap.top().second;
      heap.pop();
      std::memcpy(&rm[(size_t)i * kCols59], cur[r] + 16, kRowBytes);
      if (!push(r)) {
        cleanup();
        return io_fail("short read of the run", names[r]);
      }
      ++done;
    }
    // row-major -> column-major in 64-row tiles (cache-friendly)
    for (int64_t i0 = 0; i0 < rows_k; i0 += 64) {
      const int64_t i1 = std::min<int64_t>(rows_k, i0 + 64);
      for (int j = 0; j < kCols59; ++j)
        for (int64_t i = i0; i < i1; ++i) blk[(size_t)j * rows_k + i] = rm[(size_t)i * kCols59 + j];
    }
    const tide_status st = tide_store_put_block(res, block, blk.data());
    if (st != TIDE_OK) {
      cleanup();
      return st;
    }
    ++block;
  }
  cleanup();
  return tide_store_finalize(res);
}
