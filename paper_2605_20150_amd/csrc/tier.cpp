// Out-of-core block tier: log-structured SSD store, host LRU block cache
// with dirty bits, I/O threads, Level-1 culling, Alg. 1 residency and the
// GPU slot table, with block transfers on a side stream (Sec. 3.3 to 3.5).
#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <list>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "blocks.h"
#include "common.h"

namespace tide {
namespace {

constexpr int kCols = TIDE_D;
constexpr int64_t kPrefetchTtl = 4;   // iterations an unused prefetch is kept from other prefetches

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------- log store
// Index[k] = (file_id, offset, size, version); file 0 is the base segment,
// files >= 1 are patch segments.  An append writes the record first and
// only then moves Index[k]; the persisted index is replaced atomically
// (write, fsync, rename) at a checkpoint, so a crash during an append leaves
// the persisted Index on the previous complete version.
struct IndexEntry {
  int32_t file_id;
  int32_t pad;
  int64_t offset;
  int64_t size;
  int64_t version;
};

class LogStore {
 public:
  std::string dir;
  size_t rec = 0;
  int64_t K = 0;
  bool odirect = false;
  std::vector<IndexEntry> index;
  std::vector<int> fds;
  int64_t patch_off = 0;
  bool ready = false;   // segments created (layout build) or opened
  std::mutex mu;

  ~LogStore() {
    for (int fd : fds)
      if (fd >= 0) ::close(fd);
  }

  std::string seg_name(int id) const {
    char b[64];
    if (id == 0) return dir + "/base.seg";
    std::snprintf(b, sizeof(b), "/patch_%06d.seg", id);
    return dir + b;
  }

  int open_seg(int id, bool create) {
    int flags = O_RDWR | (create ? O_CREAT : 0);
    if (odirect) flags |= O_DIRECT;
    return ::open(seg_name(id).c_str(), flags, 0644);
  }

  tide_status create() {
    ::mkdir(dir.c_str(), 0755);
    int fd = open_seg(0, true);
    if (fd < 0) return fail("cannot create the base segment");
    // emptied first: records are written as parameters over holes (zeros)
    if (::ftruncate(fd, 0) != 0 || ::ftruncate(fd, (off_t)(rec * K)) != 0) return fail("cannot size the base segment");
    fds.assign(1, fd);
    index.resize(K);
    for (int64_t k = 0; k < K; ++k) index[k] = IndexEntry{0, 0, (int64_t)(k * rec), (int64_t)rec, 0};
    ready = true;
    return new_patch();
  }

  tide_status new_patch() {
    const int id = (int)fds.size();
    ::unlink(seg_name(id).c_str());
    int fd = open_seg(id, true);
    if (fd < 0) return fail("cannot create a patch segment");
    fds.push_back(fd);
    patch_off = 0;
    return TIDE_OK;
  }

  // With O_DIRECT every transfer goes through an aligned buffer of the
  // calling thread: pinned memory from the GPU runtime is not guaranteed to
  // be usable as the target of direct I/O.
  char* bounce() {
    thread_local std::unique_ptr<char, void (*)(void*)> buf(nullptr, std::free);
    thread_local size_t cap = 0;
    if (cap < rec) {
      void* p = nullptr;
      if (posix_memalign(&p, 4096, rec) != 0) return nullptr;
      buf.reset((char*)p);
      cap = rec;
    }
    return buf.get();
  }

  // Writes the first n bytes of block k's base record (the rest of the
  // record stays as it is: a hole, i.e. zeros, in a new base segment).
  tide_status write_base(int64_t k, const void* src, size_t n) {
    if (odirect && (reinterpret_cast<uintptr_t>(src) & 4095u) != 0) {
      char* b = bounce();
      if (!b) return fail("out of host memory for a direct-I/O buffer");
      std::memcpy(b, src, n);
      src = b;
    }
    size_t put = 0;
    while (put < n) {
      const ssize_t w = ::pwrite(fds[0], (const char*)src + put, n - put, (off_t)(k * rec + put));
      if (w <= 0) return fail("base write failed");
      put += (size_t)w;
    }
    return TIDE_OK;
  }

  tide_status read(int64_t k, void* dst) {
    IndexEntry e;
    int fd;
    {
      std::lock_guard<std::mutex> lk(mu);
      e = index[k];
      fd = fds[e.file_id];
    }
    char* to = (char*)dst;
    if (odirect && !(to = bounce())) return fail("out of host memory for a direct-I/O buffer");
    size_t got = 0;
    while (got < (size_t)e.size) {
      const ssize_t r = ::pread(fd, to + got, e.size - got, (off_t)(e.offset + got));
      if (r <= 0) return fail("segment read failed");
      got += (size_t)r;
    }
    if (to != (char*)dst) std::memcpy(dst, to, (size_t)e.size);
    return TIDE_OK;
  }

  tide_status append(int64_t k, const void* src) {
    int64_t off;
    int fid, fd;
    {
      std::lock_guard<std::mutex> lk(mu);
      off = patch_off;
      patch_off += (int64_t)rec;
      fid = (int)fds.size() - 1;
      fd = fds[fid];
    }
    if (odirect) {
      char* b = bounce();
      if (!b) return fail("out of host memory for a direct-I/O buffer");
      std::memcpy(b, src, rec);
      src = b;
    }
    size_t put = 0;
    while (put < rec) {
      const ssize_t r = ::pwrite(fd, (const char*)src + put, rec - put, (off_t)(off + put));
      if (r <= 0) return fail("patch append failed");
      put += (size_t)r;
    }
    std::lock_guard<std::mutex> lk(mu);
    index[k] = IndexEntry{fid, 0, off, (int64_t)rec, index[k].version + 1};
    return TIDE_OK;
  }

  // fsync every segment, then write the index (entries + segment count) to a
  // temporary file, fsync it and rename it over index.bin.
  tide_status persist() {
    std::vector<IndexEntry> snap;
    int nseg;
    {
      std::lock_guard<std::mutex> lk(mu);
      snap = index;
      nseg = (int)fds.size();
    }
    for (int fd : fds) ::fsync(fd);
    const std::string tmp = dir + "/index.tmp", fin = dir + "/index.bin";
    int fd = ::open(tmp.c_str(), O_WRONLY | O_CREAT | O_TRUNC, 0644);
    if (fd < 0) return fail("cannot write the index");
    const int64_t hdr[3] = {K, (int64_t)rec, nseg};
    bool ok = ::write(fd, hdr, sizeof(hdr)) == (ssize_t)sizeof(hdr);
    ok = ok && ::write(fd, snap.data(), snap.size() * sizeof(IndexEntry)) == (ssize_t)(snap.size() * sizeof(IndexEntry));
    ok = ok && ::fsync(fd) == 0;
    ::close(fd);
    if (!ok || ::rename(tmp.c_str(), fin.c_str()) != 0) return fail("index persist failed");
    int dfd = ::open(dir.c_str(), O_RDONLY);
    if (dfd >= 0) { ::fsync(dfd); ::close(dfd); }
    return TIDE_OK;
  }

  tide_status load() {
    const std::string fin = dir + "/index.bin";
    int fd = ::open(fin.c_str(), O_RDONLY);
    if (fd < 0) return fail("no persisted index in the store directory");
    int64_t hdr[3];
    bool ok = ::read(fd, hdr, sizeof(hdr)) == (ssize_t)sizeof(hdr) && hdr[0] == K && hdr[1] == (int64_t)rec;
    std::vector<IndexEntry> ix(K);
    ok = ok && ::read(fd, ix.data(), K * sizeof(IndexEntry)) == (ssize_t)(K * sizeof(IndexEntry));
    ::close(fd);
    if (!ok) return fail("persisted index does not match the configuration");
    for (int f : fds)
      if (f >= 0) ::close(f);
    fds.clear();
    for (int id = 0; id < (int)hdr[2]; ++id) {
      int f = open_seg(id, false);
      if (f < 0) return fail("missing segment file");
      fds.push_back(f);
    }
    index = ix;
    ready = true;
    return new_patch();   // later appends never touch the segments the index refers to
  }

  // Compaction (Sec. 3.4; off the training path): the current version of
  // every block is rewritten in block order into a new base segment, which
  // replaces base.seg by rename; then the Index (every entry in the new base,
  // versions kept) is persisted and the patch segments are deleted.  The
  // caller has persisted every newest version first (a checkpoint), so a
  // crash between the rename and the new Index leaves the old Index reading
  // the same versions: its base entries name records the rename did not
  // change, its patch entries patches that still exist.
  tide_status compact() {
    const std::string tmp = dir + "/base.compact";
    ::unlink(tmp.c_str());
    int fd = ::open(tmp.c_str(), O_RDWR | O_CREAT | O_TRUNC | (odirect ? O_DIRECT : 0), 0644);
    if (fd < 0) return fail("cannot create the compacted base");
    void* raw = nullptr;
    if (posix_memalign(&raw, 4096, rec) != 0) {
      ::close(fd);
      return fail("out of host memory for compaction");
    }
    std::unique_ptr<char, void (*)(void*)> buf((char*)raw, std::free);
    for (int64_t k = 0; k < K; ++k) {
      tide_status r = read(k, buf.get());
      if (r != TIDE_OK) {
        ::close(fd);
        return r;
      }
      size_t put = 0;
      while (put < rec) {
        const ssize_t w = ::pwrite(fd, buf.get() + put, rec - put, (off_t)(k * (int64_t)rec + put));
        if (w <= 0) {
          ::close(fd);
          return fail("compacted base write failed");
        }
        put += (size_t)w;
      }
    }
    const bool synced = ::fsync(fd) == 0;
    ::close(fd);
    if (!synced || ::rename(tmp.c_str(), seg_name(0).c_str()) != 0) return fail("compacted base commit failed");
    int dfd = ::open(dir.c_str(), O_RDONLY);
    if (dfd >= 0) { ::fsync(dfd); ::close(dfd); }
    const int old_nseg = (int)fds.size();
    for (int f : fds)
      if (f >= 0) ::close(f);
    fds.clear();
    const int base = open_seg(0, false);
    if (base < 0) return fail("cannot reopen the compacted base");
    fds.push_back(base);
    {
      std::lock_guard<std::mutex> lk(mu);
      for (int64_t k = 0; k < K; ++k) index[k] = IndexEntry{0, 0, (int64_t)(k * rec), (int64_t)rec, index[k].version};
    }
    tide_status r = persist();
    if (r != TIDE_OK) return r;
    for (int id = 1; id < old_nseg; ++id) ::unlink(seg_name(id).c_str());
    return new_patch();
  }

  static tide_status fail(const char* what) {
    set_error("%s (%s)", what, std::strerror(errno));
    return TIDE_EIO;
  }
};

// --------------------------------------------------------------- I/O pool
class IoPool {
 public:
  explicit IoPool(int n) {
    for (int i = 0; i < n; ++i) th_.emplace_back([this] { run(); });
  }
  ~IoPool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
  }
  // Demand work (reads the next iteration needs, write-backs) is served
  // before speculative prefetch reads; each class in FIFO order.
  void submit(std::function<void()> f, bool speculative = false) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      (speculative ? low_ : q_).push_back(std::move(f));
    }
    cv_.notify_one();
  }

 private:
  void run() {
    for (;;) {
      std::function<void()> f;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [this] { return stop_ || !q_.empty() || !low_.empty(); });
        if (stop_ && q_.empty() && low_.empty()) return;
        auto& from = q_.empty() ? low_ : q_;
        f = std::move(from.front());
        from.pop_front();
      }
      f();
    }
  }
  std::vector<std::thread> th_;
  std::deque<std::function<void()>> q_, low_;
  std::mutex mu_;
  std::condition_variable cv_;
  bool stop_ = false;
};

}  // namespace
}  // namespace tide

using namespace tide;

// ----------------------------------------------------------- the tier object
struct tide_residency {
  // configuration
  std::string dir;
  int64_t N = 0, K = 0;
  int32_t B = 0, C = 0;
  int64_t host_cap = 0;
  bool host_pool = false;
  bool no_tide = false, no_overlap = false;   // ablation switches
  bool cold_restart = false, bounded = false;  // the paper's default placement and budget
  double lambda = 0.75, gamma = 0.9, kappa = 1.32;
  size_t pbytes = 0, sbytes = 0, rec = 0;
  // caller memory
  tide_pool* pool = nullptr;
  float* d_spheres = nullptr;
  uint8_t* d_dirty = nullptr;
  // host mirrors
  std::vector<int32_t> h_slot_block, h_slot_rows, h_order;
  std::vector<float> h_spheres;
  float* h_spheres_stage = nullptr;   // pinned read-back buffers
  uint8_t* h_dirty_stage = nullptr;
  std::vector<int32_t> slot_of;       // block -> slot, -1
  std::vector<uint8_t> gpu_dirty;     // the GPU copy is newer than the host / SSD copies
  std::vector<uint8_t> ever_resident;
  std::vector<double> age;
  std::set<int32_t> R;
  std::vector<int32_t> Kcur;
  std::vector<int32_t> pending_h2d;   // S+ blocks waiting for their SSD read
  std::vector<int32_t> undecided;     // blocks copied back whose dirty flag is still in flight
  // host cache
  struct Entry {
    int64_t block = -1;
    char* buf = nullptr;
    bool valid = false, loading = false, dirty = false, flushing = false, prefetched = false;
    bool undecided = false;      // written back before its dirty flag was read; pinned until then
    bool spec_read = false;      // the pending read was queued as a speculative prefetch
    int64_t prefetch_iter = 0;   // iteration of the prefetch hint that filled the entry
    bool read_claimed = false;   // an I/O thread has started the pending read
    uint64_t read_seq = 0;       // identifies the pending read; stale queued copies skip
    hipEvent_t fence = nullptr;  // last device copy that reads or writes buf
    std::list<int>::iterator it;
  };
  std::vector<Entry> ent;
  std::unordered_map<int64_t, int> map;
  std::list<int> lru;   // front = most recently used
  std::mutex mu;
  std::condition_variable cv;
  // storage + threads
  LogStore store;
  IoPool* io = nullptr;
  tide_status io_error = TIDE_OK;
  std::string io_msg;   // message of the first failed I/O task (set on an I/O thread)
  int n_io = 1;         // I/O threads
  tide_status io_failed() const {
    set_error("block I/O failed: %s", io_msg.c_str());
    return io_error;
  }
  // device sync
  hipStream_t last_side = nullptr;
  hipEvent_t ev_compute = nullptr, ev_side = nullptr, ev_bounds = nullptr;
  std::vector<hipEvent_t> fences;
  int fence_next = 0;
  bool compute_recorded = false, bounds_pending = false;
  tide_tier_stats st{};

  char* put_buf = nullptr;   // layout-build staging record (4 KiB aligned, reused)
  ~tide_residency() {
    delete io;
    std::free(put_buf);
    for (auto& e : ent) free_host(e.buf);
    free_host((char*)h_spheres_stage);
    free_host((char*)h_dirty_stage);
    if (!host_pool) {
      for (hipEvent_t ev : fences) (void)hipEventDestroy(ev);
      if (ev_compute) (void)hipEventDestroy(ev_compute);
      if (ev_side) (void)hipEventDestroy(ev_side);
      if (ev_bounds) (void)hipEventDestroy(ev_bounds);
    }
  }

  // ---------------------------------------------------- memory helpers
  char* alloc_host(size_t n) {
    void* p = nullptr;
    if (host_pool) {
      if (posix_memalign(&p, 4096, n) != 0) return nullptr;
    } else if (hipHostMalloc(&p, n, hipHostMallocDefault) != hipSuccess) {
      return nullptr;
    }
    return (char*)p;
  }
  void free_host(char* p) {
    if (!p) return;
    if (host_pool) std::free(p);
    else (void)hipHostFree(p);
  }
  char* slot_ptr(int arr, int32_t slot) const {   // arr 0 params, 1 m, 2 v, 3 step
    if (arr == 3) return (char*)pool->step + (size_t)slot * sbytes;
    void* base = arr == 0 ? pool->params : (arr == 1 ? pool->exp_avg : pool->exp_avg_sq);
    return (char*)base + (size_t)slot * pbytes;
  }
  tide_status copy(void* dst, const void* src, size_t n, bool h2d, hipStream_t s) {
    if (host_pool) {
      std::memcpy(dst, src, n);
      return TIDE_OK;
    }
    TIDE_HIP(hipMemcpyAsync(dst, src, n, h2d ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost, s));
    return TIDE_OK;
  }
  tide_status zero(void* dst, size_t n, hipStream_t s) {
    if (host_pool) {
      std::memset(dst, 0, n);
      return TIDE_OK;
    }
    TIDE_HIP(hipMemsetAsync(dst, 0, n, s));
    return TIDE_OK;
  }
  // A cold-restart block moves its parameters only; its moments and steps
  // start from zero on the GPU.
  tide_status h2d_block(int32_t slot, const char* buf, hipStream_t s) {
    tide_status r;
    if (cold_restart) {
      if ((r = copy(slot_ptr(0, slot), buf, pbytes, true, s)) != TIDE_OK) return r;
      for (int a = 1; a < 3; ++a)
        if ((r = zero(slot_ptr(a, slot), pbytes, s)) != TIDE_OK) return r;
      if ((r = zero(slot_ptr(3, slot), sbytes, s)) != TIDE_OK) return r;
      st.h2d_bytes += (int64_t)pbytes;
      return TIDE_OK;
    }
    for (int a = 0; a < 3; ++a)
      if ((r = copy(slot_ptr(a, slot), buf + a * pbytes, pbytes, true, s)) != TIDE_OK) return r;
    if ((r = copy(slot_ptr(3, slot), buf + 3 * pbytes, sbytes, true, s)) != TIDE_OK) return r;
    st.h2d_bytes += (int64_t)rec;
    return TIDE_OK;
  }
  tide_status d2h_block(int32_t slot, char* buf, hipStream_t s) {
    tide_status r;
    const int arrays = cold_restart ? 1 : 3;
    for (int a = 0; a < arrays; ++a)
      if ((r = copy(buf + a * pbytes, slot_ptr(a, slot), pbytes, false, s)) != TIDE_OK) return r;
    if (cold_restart) {
      st.d2h_bytes += (int64_t)pbytes;
      return TIDE_OK;
    }
    if ((r = copy(buf + 3 * pbytes, slot_ptr(3, slot), sbytes, false, s)) != TIDE_OK) return r;
    st.d2h_bytes += (int64_t)rec;
    return TIDE_OK;
  }
  hipEvent_t next_fence(hipStream_t s) {
    if (host_pool) return nullptr;
    hipEvent_t ev = fences[fence_next];
    fence_next = (fence_next + 1) % (int)fences.size();
    // The slot was last recorded for a copy that many copies back, and the
    // host entry of that copy may still hold it: let that copy finish before
    // the slot is re-recorded, so a wait on the old handle never returns
    // ahead of the copy it stood for.
    (void)hipEventSynchronize(ev);
    (void)hipEventRecord(ev, s);
    return ev;
  }
  void wait_fence(Entry& e) {
    if (e.fence) {
      (void)hipEventSynchronize(e.fence);
      e.fence = nullptr;
    }
  }

  // ---------------------------------------------------- host cache
  // Returns the entry holding block k, creating it (not valid) if needed.
  // Dirty victims are handed to the I/O threads and skipped.  Called with
  // mu held.
  // A speculative caller (spec) never takes an entry filled by a recent
  // prefetch that has not been used yet.
  bool protected_prefetch(const Entry& e) const {
    return e.prefetched && st.iterations - e.prefetch_iter <= kPrefetchTtl;
  }
  int entry_for(int64_t k, std::unique_lock<std::mutex>& lk, bool spec = false) {
    auto f = map.find(k);
    if (f != map.end()) {
      lru.splice(lru.begin(), lru, ent[f->second].it);
      return f->second;
    }
    for (;;) {
      bool transient = false;   // some entry will free itself (a read or flush completes)
      for (auto it = lru.rbegin(); it != lru.rend(); ++it) {
        Entry& e = ent[*it];
        if (e.loading || e.flushing) { transient = true; continue; }
        if (e.undecided) continue;
        if (e.block >= 0 && slot_of[e.block] >= 0 && pending_contains(e.block)) { transient = true; continue; }
        if (spec && protected_prefetch(e)) continue;
        if (e.dirty) {
          start_flush(*it);
          transient = true;
          continue;
        }
        wait_fence(e);
        const int idx = *it;
        if (e.block >= 0) map.erase(e.block);
        e.block = k;
        e.valid = e.dirty = e.prefetched = false;
        map[k] = idx;
        lru.splice(lru.begin(), lru, e.it);
        return idx;
      }
      if (io_error != TIDE_OK) return -1;
      if (!transient) {
        // every entry is pinned until the next sync_bounds: waiting would never end
        set_error("host cache of %lld blocks too small: every entry holds a block of the iteration in flight",
                  (long long)host_cap);
        return -1;
      }
      cv.wait(lk);   // every entry is busy: wait for a read or flush to finish
    }
  }
  // status of a failed entry_for
  tide_status no_entry() const { return io_error != TIDE_OK ? io_failed() : TIDE_ECAPACITY; }
  bool pending_contains(int64_t k) const {
    return std::find(pending_h2d.begin(), pending_h2d.end(), (int32_t)k) != pending_h2d.end();
  }
  void start_flush(int idx) {
    Entry& e = ent[idx];
    wait_fence(e);
    e.flushing = true;
    const int64_t blk = e.block;
    char* buf = e.buf;
    io->submit([this, idx, blk, buf] {
      const tide_status r = store.append(blk, buf);
      std::lock_guard<std::mutex> g(mu);
      if (r != TIDE_OK && io_error == TIDE_OK) { io_error = r; io_msg = tide_last_error(); }
      st.ssd_write_bytes += (int64_t)rec;
      ent[idx].flushing = false;
      ent[idx].dirty = false;
      cv.notify_all();
    });
  }
  // A read of entry idx's block into its buffer.  The same read may be queued
  // twice (a prefetch promoted to demand priority); the first copy to run
  // claims it and the other, or any copy left from an older read of the
  // entry, does nothing.
  std::function<void()> read_task(int idx, uint64_t seq, int64_t blk, char* buf) {
    return [this, idx, seq, blk, buf] {
      {
        std::lock_guard<std::mutex> g(mu);
        if (ent[idx].read_seq != seq || ent[idx].read_claimed || !ent[idx].loading) return;
        ent[idx].read_claimed = true;
      }
      const tide_status r = store.read(blk, buf);
      std::lock_guard<std::mutex> g(mu);
      if (r != TIDE_OK && io_error == TIDE_OK) { io_error = r; io_msg = tide_last_error(); }
      st.ssd_read_bytes += (int64_t)rec;
      ent[idx].loading = false;
      ent[idx].valid = true;
      if (r == TIDE_OK) issue_pending(idx);
      cv.notify_all();
    };
  }
  // A block that the last delta admitted while its SSD read was still running
  // goes host -> GPU on that delta's side stream as soon as the read is done
  // (called with mu held).  The side stream orders it after the delta's
  // write-back copies, which may have used the same slot.
  void issue_pending(int idx) {
    Entry& e = ent[idx];
    const int32_t k = (int32_t)e.block;
    auto it = std::find(pending_h2d.begin(), pending_h2d.end(), k);
    if (it == pending_h2d.end()) return;
    pending_h2d.erase(it);
    if (k < 0 || slot_of[k] < 0) return;
    const tide_status r = h2d_block(slot_of[k], e.buf, last_side);
    if (r != TIDE_OK) {
      if (io_error == TIDE_OK) { io_error = r; io_msg = tide_last_error(); }
      return;
    }
    e.fence = next_fence(last_side);
  }
  void start_read(int idx, bool speculative = false) {
    Entry& e = ent[idx];
    e.loading = true;
    e.read_claimed = false;
    e.spec_read = speculative;
    ++e.read_seq;
    io->submit(read_task(idx, e.read_seq, e.block, e.buf), speculative);
  }
  // A pending prefetch read that is now needed moves to demand priority.
  void promote(int idx) {
    Entry& e = ent[idx];
    if (!e.loading || !e.spec_read || e.read_claimed) return;
    e.spec_read = false;
    io->submit(read_task(idx, e.read_seq, e.block, e.buf), false);
  }
  // Entry for block k with its newest data, reading from the SSD if needed
  // (blocking).  Counts a hit or a miss.
  int fetch_blocking(int64_t k, std::unique_lock<std::mutex>& lk) {
    const int idx = entry_for(k, lk);
    if (idx < 0) return -1;
    Entry& e = ent[idx];
    if (e.valid || e.loading) st.host_hits++;
    else { st.host_misses++; start_read(idx); }
    promote(idx);
    cv.wait(lk, [&] { return !ent[idx].loading; });
    if (ent[idx].prefetched) { st.prefetch_used++; ent[idx].prefetched = false; }
    wait_fence(ent[idx]);   // a write-back copy into this entry may still be in flight on another stream
    return idx;
  }

  // ---------------------------------------------------- slots
  int32_t free_slot() const {
    for (int32_t s = 0; s < (int32_t)h_slot_block.size(); ++s)
      if (h_slot_block[s] < 0) return s;
    return -1;
  }
  void occupy(int32_t slot, int64_t k) {
    h_slot_block[slot] = (int32_t)k;
    h_slot_rows[slot] = (int32_t)std::min<int64_t>(B, N - k * (int64_t)B);
    slot_of[k] = slot;
    if (ever_resident[k]) st.readmissions++;
    ever_resident[k] = 1;
  }
  void release(int32_t slot) {
    const int32_t k = h_slot_block[slot];
    if (k >= 0) slot_of[k] = -1;
    h_slot_block[slot] = -1;
    h_slot_rows[slot] = 0;
  }
  tide_status upload_tables(hipStream_t s) {
    tide_status r;
    const size_t n = h_slot_block.size() * sizeof(int32_t);
    if ((r = copy((void*)pool->slot_block, h_slot_block.data(), n, true, s)) != TIDE_OK) return r;
    if ((r = copy((void*)pool->slot_rows, h_slot_rows.data(), n, true, s)) != TIDE_OK) return r;
    if (!h_order.empty() &&
        (r = copy((void*)pool->order, h_order.data(), h_order.size() * sizeof(int32_t), true, s)) != TIDE_OK)
      return r;
    pool->n_order = (int32_t)h_order.size();
    // the tables are pageable host vectors: finish the copies before they change
    if (!host_pool) TIDE_HIP(hipStreamSynchronize(s));
    return TIDE_OK;
  }

  // Evicts block k (resident): copies it back into the host cache when the
  // GPU copy may be newer, then frees its slot.  Copies go on stream s.  A
  // block of the current K_t may have been updated by the iteration still in
  // flight: it is copied back and its entry stays "undecided" (pinned) until
  // tide_residency_sync_bounds reads that iteration's dirty flags.
  tide_status evict(int64_t k, hipStream_t s, std::unique_lock<std::mutex>& lk) {
    const int32_t slot = slot_of[k];
    const bool in_flight = std::binary_search(Kcur.begin(), Kcur.end(), (int32_t)k);
    if (gpu_dirty[k] || in_flight) {
      const int idx = entry_for(k, lk);
      if (idx < 0) return no_entry();
      Entry& e = ent[idx];
      cv.wait(lk, [&] { return !ent[idx].loading && !ent[idx].flushing; });
      tide_status r = d2h_block(slot, e.buf, s);
      if (r != TIDE_OK) return r;
      e.fence = next_fence(s);
      e.valid = true;
      if (gpu_dirty[k]) {
        e.dirty = true;
      } else {
        e.undecided = true;
        undecided.push_back((int32_t)k);
      }
      gpu_dirty[k] = 0;
    }
    release(slot);
    R.erase((int32_t)k);
    st.blocks_out++;
    return TIDE_OK;
  }
};

// =========================================================================
extern "C" {

size_t tide_block_record_bytes(int32_t block_rows) {
  return (size_t)block_rows * (3 * kCols * sizeof(float) + sizeof(uint32_t));
}

tide_status tide_residency_create(const tide_store_cfg* cfg, tide_pool* pool, float* d_spheres, uint8_t* d_dirty,
                                  tide_residency** out) {
  TIDE_CHECK_ARG(cfg && pool && d_spheres && d_dirty && out && cfg->dir, "null argument");
  TIDE_CHECK_ARG(cfg->n_rows > 0 && cfg->block_rows > 0 && pool->block_rows == cfg->block_rows,
                 "block_rows must match the pool");
  TIDE_CHECK_ARG(pool->dtype == TIDE_F32, "the tier stores f32 pools");
  TIDE_CHECK_ARG(cfg->capacity > 0 && cfg->capacity <= pool->n_slots, "capacity must be in [1, n_slots]");
  TIDE_CHECK_ARG(cfg->host_cache_blocks >= 4, "host cache needs at least 4 blocks");
  TIDE_CHECK_ARG(cfg->io_threads >= 1 && cfg->io_threads <= 64, "io_threads in [1, 64]");
  TIDE_CHECK_ARG(cfg->lambda_ >= 0 && cfg->lambda_ <= 1 && cfg->gamma > 0 && cfg->gamma <= 1, "bad lambda / gamma");
  TIDE_CHECK_ARG(pool->params && pool->exp_avg && pool->exp_avg_sq && pool->step && pool->slot_block &&
                     pool->slot_rows && pool->order,
                 "pool has a null pointer");
  const bool odirect = (cfg->flags & TIDE_TIER_ODIRECT) != 0;
  TIDE_CHECK_ARG(!odirect || cfg->block_rows % 512 == 0, "O_DIRECT needs block_rows to be a multiple of 512");
  auto* r = new tide_residency();
  r->dir = cfg->dir;
  r->N = cfg->n_rows;
  r->B = cfg->block_rows;
  r->K = (cfg->n_rows + cfg->block_rows - 1) / cfg->block_rows;
  r->C = cfg->capacity;
  r->host_cap = cfg->host_cache_blocks;
  r->host_pool = (cfg->flags & TIDE_TIER_HOST_POOL) != 0;
  r->no_tide = (cfg->flags & TIDE_TIER_NO_TIDE) != 0;
  r->no_overlap = (cfg->flags & TIDE_TIER_NO_OVERLAP) != 0;
  r->cold_restart = (cfg->flags & TIDE_TIER_COLD_RESTART) != 0;
  r->bounded = (cfg->flags & TIDE_TIER_BOUNDED) != 0;
  r->lambda = cfg->lambda_;
  r->gamma = cfg->gamma;
  r->kappa = cfg->kappa;
  r->pbytes = (size_t)kCols * r->B * sizeof(float);
  r->sbytes = (size_t)r->B * sizeof(uint32_t);
  r->rec = tide_block_record_bytes(r->B);
  r->pool = pool;
  r->d_spheres = d_spheres;
  r->d_dirty = d_dirty;
  r->h_slot_block.assign(pool->n_slots, -1);
  r->h_slot_rows.assign(pool->n_slots, 0);
  r->h_spheres.assign(4 * r->K, 0.f);
  r->slot_of.assign(r->K, -1);
  r->gpu_dirty.assign(r->K, 0);
  r->ever_resident.assign(r->K, 0);
  r->age.assign(r->K, 1e9);
  r->store.dir = r->dir;
  r->store.rec = r->rec;
  r->store.K = r->K;
  r->store.odirect = odirect;
  r->ent.resize(r->host_cap);
  for (int64_t i = 0; i < r->host_cap; ++i) {
    r->ent[i].buf = r->alloc_host(r->rec);
    if (!r->ent[i].buf) {
      delete r;
      set_error("cannot allocate %lld host cache blocks of %zu bytes", (long long)cfg->host_cache_blocks,
                tide_block_record_bytes(cfg->block_rows));
      return TIDE_ECAPACITY;
    }
    r->lru.push_back((int)i);
    r->ent[i].it = std::prev(r->lru.end());
  }
  r->h_spheres_stage = (float*)r->alloc_host(std::max<size_t>(16 * r->K, 16));
  r->h_dirty_stage = (uint8_t*)r->alloc_host(std::max<size_t>(r->K, 16));
  if (!r->h_spheres_stage || !r->h_dirty_stage) {
    delete r;
    set_error("cannot allocate the read-back buffers");
    return TIDE_ECAPACITY;
  }
  if (!r->host_pool) {
    r->fences.resize(64);
    for (auto& ev : r->fences) (void)hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    (void)hipEventCreateWithFlags(&r->ev_compute, hipEventDisableTiming);
    (void)hipEventCreateWithFlags(&r->ev_side, hipEventDisableTiming);
    (void)hipEventCreateWithFlags(&r->ev_bounds, hipEventDisableTiming);
  }
  r->io = new IoPool(cfg->io_threads);
  r->n_io = cfg->io_threads;
  *out = r;
  return TIDE_OK;
}

tide_status tide_residency_destroy(tide_residency* res) {
  if (!res) return TIDE_OK;
  {
    std::unique_lock<std::mutex> lk(res->mu);
    res->cv.wait(lk, [&] {
      for (auto& e : res->ent)
        if (e.loading || e.flushing) return false;
      return true;
    });
  }
  delete res;
  return TIDE_OK;
}

tide_status tide_store_put_block(tide_residency* res, int64_t block, const float* params) {
  TIDE_CHECK_ARG(res && params, "null argument");
  TIDE_CHECK_ARG(block >= 0 && block < res->K, "block out of range");
  if (!res->store.ready) {
    const tide_status c = res->store.create();
    if (c != TIDE_OK) return c;
  }
  const int64_t rows = std::min<int64_t>(res->B, res->N - block * (int64_t)res->B);
  // one 4 KiB-aligned record reused across blocks (written directly with
  // O_DIRECT); moments and steps stay zero, the column tails are cleared
  if (!res->put_buf) {
    void* raw = nullptr;
    if (posix_memalign(&raw, 4096, res->rec) != 0) return LogStore::fail("out of host memory for the layout build");
    res->put_buf = (char*)raw;
    std::memset(res->put_buf, 0, res->rec);
  }
  float* P = (float*)res->put_buf;
  for (int j = 0; j < kCols; ++j) {
    std::memcpy(P + (size_t)j * res->B, params + (size_t)j * rows, rows * sizeof(float));
    if (rows < res->B) std::memset(P + (size_t)j * res->B + rows, 0, (size_t)(res->B - rows) * sizeof(float));
  }
  block_sphere(P, res->B, rows, res->kappa, &res->h_spheres[4 * block]);
  // zero moments and steps are the new base segment's holes: only the
  // parameters are written (a third of the record)
  return res->store.write_base(block, res->put_buf, res->pbytes);
}

static tide_status upload_spheres(tide_residency* res) {
  std::memcpy(res->h_spheres_stage, res->h_spheres.data(), 16 * res->K);
  if (res->host_pool) {
    std::memcpy(res->d_spheres, res->h_spheres_stage, 16 * res->K);
    std::memset(res->d_dirty, 0, res->K);
    return TIDE_OK;
  }
  TIDE_HIP(hipMemcpy(res->d_spheres, res->h_spheres_stage, 16 * res->K, hipMemcpyHostToDevice));
  std::memset(res->h_dirty_stage, 0, res->K);
  TIDE_HIP(hipMemcpy(res->d_dirty, res->h_dirty_stage, res->K, hipMemcpyHostToDevice));
  return TIDE_OK;
}

static tide_status write_sphere_file(tide_residency* res) {
  const std::string p = res->dir + "/spheres.bin";
  FILE* f = std::fopen(p.c_str(), "wb");
  if (!f) return LogStore::fail("cannot write spheres.bin");
  const bool ok = std::fwrite(res->h_spheres.data(), 4, res->h_spheres.size(), f) == res->h_spheres.size();
  std::fclose(f);
  return ok ? TIDE_OK : LogStore::fail("cannot write spheres.bin");
}

tide_status tide_store_finalize(tide_residency* res) {
  TIDE_CHECK_ARG(res, "null argument");
  TIDE_CHECK_ARG(res->store.ready, "no block was written");
  tide_status s;
  if ((s = res->store.persist()) != TIDE_OK) return s;
  if ((s = write_sphere_file(res)) != TIDE_OK) return s;
  return upload_spheres(res);
}

tide_status tide_store_open(tide_residency* res) {
  TIDE_CHECK_ARG(res, "null argument");
  tide_status s;
  if ((s = res->store.load()) != TIDE_OK) return s;
  const std::string p = res->dir + "/spheres.bin";
  FILE* f = std::fopen(p.c_str(), "rb");
  if (!f) return LogStore::fail("missing spheres.bin");
  const bool ok = std::fread(res->h_spheres.data(), 4, res->h_spheres.size(), f) == res->h_spheres.size();
  std::fclose(f);
  if (!ok) return LogStore::fail("short spheres.bin");
  return upload_spheres(res);
}

// Level 1 (Sec. 3.3), per camera (CullCam).
tide_status tide_cull_blocks(const tide_residency* res, const tide_camera* cams, int32_t n_cams, int32_t* out_ids,
                             int32_t* counts, int64_t cap) {
  TIDE_CHECK_ARG(res && cams && out_ids && counts, "null argument");
  TIDE_CHECK_ARG(n_cams >= 1 && n_cams <= TIDE_MAX_CAMS, "bad n_cams");
  int64_t n = 0;
  for (int ci = 0; ci < n_cams; ++ci) {
    const CullCam cc(cams[ci]);
    int32_t cnt = 0;
    for (int64_t k = 0; k < res->K; ++k) {
      if (!cc.keep(&res->h_spheres[4 * k])) continue;
      if (n >= cap) {
        set_error("cull output capacity %lld exceeded", (long long)cap);
        return TIDE_ECAPACITY;
      }
      out_ids[n++] = (int32_t)k;
      ++cnt;
    }
    counts[ci] = cnt;
  }
  return TIDE_OK;
}

tide_status tide_ensure_resident(tide_residency* res, const int32_t* K, int32_t n, void* compute_stream,
                                 double* stall_s) {
  TIDE_CHECK_ARG(res && (K || n == 0) && n >= 0, "null argument");
  TIDE_CHECK_ARG(res->bounded || n <= res->pool->n_slots, "K_t (%d blocks) exceeds the pool's %d slots", n,
                 res->pool->n_slots);
  hipStream_t cs = (hipStream_t)compute_stream;
  const double t0 = now_s();
  std::unique_lock<std::mutex> lk(res->mu);
  if (res->io_error != TIDE_OK) return res->io_failed();
  std::vector<int32_t> need(K, K + n);
  std::sort(need.begin(), need.end());
  need.erase(std::unique(need.begin(), need.end()), need.end());
  for (int32_t k : need) TIDE_CHECK_ARG(k >= 0 && k < res->K, "block id %d out of range", k);
  const std::set<int32_t> want(need.begin(), need.end());
  bool copied = false;
  // S+ blocks of K_t whose SSD read is still running: the read completes and
  // issues their copy on the side stream; wait (host) for that
  for (int32_t k : need) {
    if (res->slot_of[k] < 0 || !res->pending_contains(k)) continue;
    const auto f = res->map.find(k);
    if (f != res->map.end()) res->promote(f->second);
    res->cv.wait(lk, [&] { return !res->pending_contains(k) || res->io_error != TIDE_OK; });
    if (res->io_error != TIDE_OK) return res->io_failed();
  }
  // blocks of K_t that are not resident at all: synchronous fetch (or, under
  // a binding budget, left out of this render)
  if (res->bounded) {
    std::vector<int32_t> kept;
    for (int32_t k : need)
      if (res->slot_of[k] >= 0) kept.push_back(k);
    res->st.skipped += (int64_t)(need.size() - kept.size());
    need.swap(kept);
  }
  for (int32_t k : need) {
    if (res->slot_of[k] >= 0) continue;
    int32_t slot = res->free_slot();
    if (slot < 0) {
      // evict the resident block outside K_t that Alg. 1 scores lowest
      int32_t victim = -1;
      double best = 1e300;
      for (int32_t b : res->R) {
        if (want.count(b)) continue;
        const double sc = std::pow(res->gamma, res->age[b]);
        if (sc < best || (sc == best && b > victim)) { best = sc; victim = b; }
      }
      if (victim < 0) {
        set_error("no slot available for a block of K_t");
        return TIDE_ECAPACITY;
      }
      const int32_t vs = res->slot_of[victim];
      tide_status r = res->evict(victim, cs, lk);
      if (r != TIDE_OK) return r;
      slot = vs;
    }
    const int idx = res->fetch_blocking(k, lk);
    if (idx < 0) return res->no_entry();
    res->occupy(slot, k);
    res->R.insert(k);
    tide_status r = res->h2d_block(slot, res->ent[idx].buf, cs);
    if (r != TIDE_OK) return r;
    res->ent[idx].fence = res->next_fence(cs);
    res->st.sync_fetches++;
    copied = true;
  }
  // the compute waits for every side-stream transfer issued so far (the
  // last delta's copies and the completed reads' copies)
  if (!res->host_pool && res->last_side) {
    TIDE_HIP(hipEventRecord(res->ev_side, res->last_side));
    TIDE_HIP(hipStreamWaitEvent(cs, res->ev_side, 0));
  }
  lk.unlock();
  if (copied && !res->host_pool) TIDE_HIP(hipStreamSynchronize(cs));
  // render order: slots of K_t by ascending block id (pidx order = global-id order)
  res->h_order.clear();
  for (int32_t k : need) res->h_order.push_back(res->slot_of[k]);
  res->Kcur = need;
  tide_status r = res->upload_tables(cs);
  if (r != TIDE_OK) return r;
  const double stall = now_s() - t0;
  res->st.stall_seconds += stall;
  if (stall_s) *stall_s = stall;
  res->st.resident = (int64_t)res->R.size();
  return TIDE_OK;
}

tide_status tide_residency_end_iteration(tide_residency* res, void* compute_stream) {
  TIDE_CHECK_ARG(res, "null argument");
  hipStream_t cs = (hipStream_t)compute_stream;
  res->st.iterations++;
  if (res->host_pool) {
    std::memcpy(res->h_spheres_stage, res->d_spheres, 16 * res->K);
    std::memcpy(res->h_dirty_stage, res->d_dirty, res->K);
    std::memset(res->d_dirty, 0, res->K);
    res->bounds_pending = true;
    res->compute_recorded = true;
    return TIDE_OK;
  }
  TIDE_HIP(hipEventRecord(res->ev_compute, cs));
  res->compute_recorded = true;
  TIDE_HIP(hipMemcpyAsync(res->h_spheres_stage, res->d_spheres, 16 * res->K, hipMemcpyDeviceToHost, cs));
  TIDE_HIP(hipMemcpyAsync(res->h_dirty_stage, res->d_dirty, res->K, hipMemcpyDeviceToHost, cs));
  TIDE_HIP(hipMemsetAsync(res->d_dirty, 0, res->K, cs));
  TIDE_HIP(hipEventRecord(res->ev_bounds, cs));
  res->bounds_pending = true;
  return TIDE_OK;
}

tide_status tide_residency_sync_bounds(tide_residency* res) {
  TIDE_CHECK_ARG(res, "null argument");
  if (!res->bounds_pending) return TIDE_OK;
  if (!res->host_pool) TIDE_HIP(hipEventSynchronize(res->ev_bounds));
  std::memcpy(res->h_spheres.data(), res->h_spheres_stage, 16 * res->K);
  std::lock_guard<std::mutex> lk(res->mu);
  // blocks copied back during the iteration: their entries are dirty iff the
  // iteration updated them
  for (int32_t k : res->undecided) {
    auto f = res->map.find(k);
    if (f == res->map.end()) continue;
    auto& e = res->ent[f->second];
    if (res->h_dirty_stage[k]) e.dirty = true;
    e.undecided = false;
  }
  res->undecided.clear();
  for (int64_t k = 0; k < res->K; ++k)
    if (res->h_dirty_stage[k] && res->slot_of[k] >= 0) res->gpu_dirty[k] = 1;
  res->bounds_pending = false;
  res->cv.notify_all();
  return TIDE_OK;
}

// Alg. 1 (Sec. 3.5): recency update, residency score, camera-balanced Top-C,
// set differences; then the transfers.
tide_status tide_stream_delta(tide_residency* res, const int32_t* knext_ids, const int32_t* knext_counts,
                              int32_t n_cams, void* side_stream, int32_t* out_plus, int32_t* n_plus,
                              int32_t* out_minus, int32_t* n_minus, int64_t cap) {
  TIDE_CHECK_ARG(res && knext_counts && n_cams >= 1 && n_cams <= TIDE_MAX_CAMS, "bad arguments");
  hipStream_t ss = (hipStream_t)side_stream;
  std::unique_lock<std::mutex> lk(res->mu);
  if (res->io_error != TIDE_OK) return res->io_failed();
  // 1. next working set, per camera and united
  std::vector<std::vector<int32_t>> Kj(n_cams);
  std::set<int32_t> Kn;
  int64_t off = 0;
  for (int j = 0; j < n_cams; ++j) {
    TIDE_CHECK_ARG(knext_counts[j] >= 0, "negative count");
    for (int32_t i = 0; i < knext_counts[j]; ++i) {
      const int32_t k = knext_ids[off + i];
      TIDE_CHECK_ARG(k >= 0 && k < res->K, "block id out of range");
      Kj[j].push_back(k);
      Kn.insert(k);
    }
    off += knext_counts[j];
  }
  // 2. recency: age 0 for the accessed resident blocks R_t intersect K_t.
  //    The new ages are kept aside and stored only once the call can no
  //    longer fail, so a rejected call leaves the tier's state unchanged.
  std::vector<double> age(res->K);
  {
    std::vector<uint8_t> acc(res->K, 0);
    for (int32_t k : res->Kcur)
      if (res->R.count(k)) acc[k] = 1;
    for (int64_t k = 0; k < res->K; ++k) age[k] = acc[k] ? 0.0 : res->age[k] + 1.0;
  }
  // 3.-5. candidates, scores, camera-balanced Top-C
  std::set<int32_t> Ct = res->R;
  Ct.insert(Kn.begin(), Kn.end());
  const double lam = res->lambda, gam = res->gamma;
  auto score = [&](int32_t k) { return lam * (Kn.count(k) ? 1.0 : 0.0) + (1.0 - lam) * std::pow(gam, age[k]); };
  auto better = [&](int32_t a, int32_t b) {
    const double sa = score(a), sb = score(b);
    return sa != sb ? sa > sb : a < b;
  };
  std::set<int32_t> chosen;
  const int q = res->C / (4 * n_cams);
  for (int j = 0; j < n_cams; ++j) {
    std::vector<int32_t> cand;
    for (int32_t k : Kj[j])
      if (!chosen.count(k)) cand.push_back(k);
    std::sort(cand.begin(), cand.end());
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    std::stable_sort(cand.begin(), cand.end(), better);
    for (int i = 0; i < (int)cand.size() && i < q && (int)chosen.size() < res->C; ++i) chosen.insert(cand[i]);
  }
  std::vector<int32_t> rest;
  for (int32_t k : Ct)
    if (!chosen.count(k)) rest.push_back(k);
  std::stable_sort(rest.begin(), rest.end(), better);
  for (size_t i = 0; i < rest.size() && (int)chosen.size() < res->C; ++i) chosen.insert(rest[i]);
  // 6. set differences (the no-Tide ablation moves all of K_{t+1} again and
  //    lets every resident block go)
  std::vector<int32_t> Sp, Sm;
  if (res->no_tide) {
    // blocks that are not resident first: they can take free slots at once
    TIDE_CHECK_ARG((int64_t)Kn.size() <= res->C, "K_{t+1} (%zu blocks) exceeds the capacity", Kn.size());
    for (int32_t k : Kn)
      if (!res->R.count(k)) Sp.push_back(k);
    for (int32_t k : Kn)
      if (res->R.count(k)) Sp.push_back(k);
    Sm.assign(res->R.begin(), res->R.end());
  } else {
    for (int32_t k : chosen)
      if (!res->R.count(k)) Sp.push_back(k);
    for (int32_t k : res->R)
      if (!chosen.count(k)) Sm.push_back(k);
  }
  if (out_plus) TIDE_CHECK_ARG((int64_t)Sp.size() <= cap, "S+ (%zu blocks) exceeds the output capacity %lld", Sp.size(),
                               (long long)cap);
  if (out_minus) TIDE_CHECK_ARG((int64_t)Sm.size() <= cap, "S- (%zu blocks) exceeds the output capacity %lld",
                                Sm.size(), (long long)cap);
  res->age.swap(age);
  if (n_plus) *n_plus = (int32_t)Sp.size();
  if (n_minus) *n_minus = (int32_t)Sm.size();
  if (out_plus) std::copy(Sp.begin(), Sp.end(), out_plus);
  if (out_minus) std::copy(Sm.begin(), Sm.end(), out_minus);
  res->st.blocks_in += (int64_t)Sp.size();

  // transfers.  S+ blocks (ascending id) first take slots nobody holds (their
  // copies overlap the current compute), then the slots S- frees (after the
  // current compute and the write-back copies).  A block whose data is not in
  // the host cache yet gets an SSD read and its copy is left for
  // tide_ensure_resident.
  std::vector<int32_t> free_now;
  for (int32_t s = 0; s < (int32_t)res->h_slot_block.size(); ++s)
    if (res->h_slot_block[s] < 0) free_now.push_back(s);
  size_t next = 0;
  auto admit = [&](int32_t k, int32_t slot) -> tide_status {
    res->occupy(slot, k);
    res->R.insert(k);
    const int idx = res->entry_for(k, lk);
    if (idx < 0) return res->no_entry();
    auto& e = res->ent[idx];
    if (e.valid && !e.loading) {
      res->st.host_hits++;
      if (e.prefetched) { res->st.prefetch_used++; e.prefetched = false; }
      tide_status r = res->h2d_block(slot, e.buf, ss);
      if (r != TIDE_OK) return r;
      e.fence = res->next_fence(ss);
    } else {
      if (!e.loading) { res->st.host_misses++; res->start_read(idx); }
      else if (e.prefetched) { res->st.prefetch_used++; e.prefetched = false; }
      res->promote(idx);
      if (!res->pending_contains(k)) res->pending_h2d.push_back(k);
    }
    return TIDE_OK;
  };
  const double t_serial = now_s();
  if (res->no_overlap && !res->host_pool && res->compute_recorded) TIDE_HIP(hipEventSynchronize(res->ev_compute));
  size_t i = 0;
  // (with no_tide a resident block leaves and comes back in the same delta:
  // its admission waits for its eviction)
  for (; i < Sp.size() && next < free_now.size() && !(res->no_tide && res->R.count(Sp[i])); ++i) {
    tide_status r = admit(Sp[i], free_now[next++]);
    if (r != TIDE_OK) return r;
  }
  if (!res->host_pool && !Sm.empty() && res->compute_recorded) TIDE_HIP(hipStreamWaitEvent(ss, res->ev_compute, 0));
  std::vector<int32_t> freed;
  for (int32_t k : Sm) {
    const int32_t slot = res->slot_of[k];
    tide_status r = res->evict(k, ss, lk);
    if (r != TIDE_OK) return r;
    freed.push_back(slot);
  }
  if (res->no_tide) freed.insert(freed.end(), free_now.begin() + (std::ptrdiff_t)next, free_now.end());
  std::sort(freed.begin(), freed.end());
  for (size_t f = 0; i < Sp.size() && f < freed.size(); ++i, ++f) {
    tide_status r = admit(Sp[i], freed[f]);
    if (r != TIDE_OK) return r;
  }
  if (i < Sp.size()) {
    set_error("internal: S+ larger than the free slots");
    return TIDE_ESTATE;
  }
  if (!res->host_pool) TIDE_HIP(hipEventRecord(res->ev_side, ss));
  res->last_side = ss;
  res->st.resident = (int64_t)res->R.size();
  if (res->no_overlap) {
    // serialised: every read and copy of this delta completes before the
    // next compute can be enqueued
    res->cv.wait(lk, [&] { return res->pending_h2d.empty() || res->io_error != TIDE_OK; });
    if (res->io_error != TIDE_OK) return res->io_failed();
    if (!res->host_pool) TIDE_HIP(hipStreamSynchronize(ss));
    res->st.stall_seconds += now_s() - t_serial;
  }
  return TIDE_OK;
}

tide_status tide_prefetch_hint(tide_residency* res, const int32_t* blocks, int32_t n, int32_t horizon) {
  TIDE_CHECK_ARG(res && (blocks || n == 0), "null argument");
  (void)horizon;
  std::unique_lock<std::mutex> lk(res->mu);
  int outstanding = 0;
  for (const auto& e : res->ent) outstanding += (e.loading && e.spec_read) ? 1 : 0;
  const int cap = 2 * res->n_io;
  for (int32_t i = 0; i < n && outstanding < cap; ++i) {
    const int32_t k = blocks[i];
    TIDE_CHECK_ARG(k >= 0 && k < res->K, "block id out of range");
    if (res->slot_of[k] >= 0 || res->map.count(k)) continue;
    // only a clean, idle entry that no recent prefetch filled may be given up
    bool room = false;
    for (auto it = res->lru.rbegin(); it != res->lru.rend(); ++it) {
      auto& e = res->ent[*it];
      if (!e.loading && !e.flushing && !e.dirty && !e.undecided && !res->protected_prefetch(e) &&
          !(e.block >= 0 && res->pending_contains(e.block))) {
        room = true;
        break;
      }
    }
    if (!room) break;
    const int idx = res->entry_for(k, lk, true);
    if (idx < 0) return res->no_entry();
    res->ent[idx].prefetched = true;
    res->ent[idx].prefetch_iter = res->st.iterations;
    res->start_read(idx, true);
    res->st.prefetch_issued++;
    ++outstanding;
  }
  if (res->no_overlap) {
    // serialised: the read-ahead also completes before the next compute
    const double t0 = now_s();
    res->cv.wait(lk, [&] {
      if (res->io_error != TIDE_OK) return true;
      for (const auto& e : res->ent)
        if (e.loading && e.spec_read) return false;
      return true;
    });
    res->st.stall_seconds += now_s() - t0;
    if (res->io_error != TIDE_OK) return res->io_failed();
  }
  return TIDE_OK;
}

tide_status tide_checkpoint(tide_residency* res) {
  TIDE_CHECK_ARG(res, "null argument");
  tide_status r = tide_residency_sync_bounds(res);
  if (r != TIDE_OK) return r;
  std::unique_lock<std::mutex> lk(res->mu);
  // dirty GPU blocks -> host cache (dirty)
  for (int32_t k : res->R) {
    if (!res->gpu_dirty[k]) continue;
    const int idx = res->entry_for(k, lk);
    if (idx < 0) return res->no_entry();
    res->cv.wait(lk, [&] { return !res->ent[idx].loading && !res->ent[idx].flushing; });
    if (res->host_pool) {
      r = res->d2h_block(res->slot_of[k], res->ent[idx].buf, nullptr);
    } else {
      lk.unlock();
      r = res->d2h_block(res->slot_of[k], res->ent[idx].buf, nullptr);
      if (r == TIDE_OK && hipStreamSynchronize(nullptr) != hipSuccess) r = TIDE_EHIP;
      lk.lock();
    }
    if (r != TIDE_OK) return r;
    res->ent[idx].valid = true;
    res->ent[idx].dirty = true;
    res->gpu_dirty[k] = 0;
  }
  // flush every dirty host entry, then persist the index
  for (size_t i = 0; i < res->ent.size(); ++i)
    if (res->ent[i].dirty && !res->ent[i].flushing) res->start_flush((int)i);
  res->cv.wait(lk, [&] {
    for (auto& e : res->ent)
      if (e.flushing) return false;
    return true;
  });
  if (res->io_error != TIDE_OK) return res->io_failed();
  lk.unlock();
  r = res->store.persist();
  if (r != TIDE_OK) return r;
  return write_sphere_file(res);
}

tide_status tide_store_compact(tide_residency* res) {
  TIDE_CHECK_ARG(res, "null argument");
  tide_status r = tide_checkpoint(res);
  if (r != TIDE_OK) return r;
  std::unique_lock<std::mutex> lk(res->mu);
  // no read or write-back may touch the segments meanwhile
  res->cv.wait(lk, [&] {
    if (res->io_error != TIDE_OK) return true;
    for (const auto& e : res->ent)
      if (e.loading || e.flushing || e.dirty) return false;
    return true;
  });
  if (res->io_error != TIDE_OK) return res->io_failed();
  return res->store.compact();
}

tide_status tide_read_block(tide_residency* res, int64_t block, void* dst) {
  TIDE_CHECK_ARG(res && dst && block >= 0 && block < res->K, "bad arguments");
  std::unique_lock<std::mutex> lk(res->mu);
  const int32_t slot = res->slot_of[block];
  // a slot whose copy is still waiting for the SSD read does not hold the block yet
  if (slot >= 0 && !res->pending_contains(block)) {
    lk.unlock();
    if (!res->host_pool) TIDE_HIP(hipDeviceSynchronize());
    char* d = (char*)dst;
    for (int a = 0; a < 3; ++a) {
      if (res->host_pool) std::memcpy(d + a * res->pbytes, res->slot_ptr(a, slot), res->pbytes);
      else TIDE_HIP(hipMemcpy(d + a * res->pbytes, res->slot_ptr(a, slot), res->pbytes, hipMemcpyDeviceToHost));
    }
    if (res->host_pool) std::memcpy(d + 3 * res->pbytes, res->slot_ptr(3, slot), res->sbytes);
    else TIDE_HIP(hipMemcpy(d + 3 * res->pbytes, res->slot_ptr(3, slot), res->sbytes, hipMemcpyDeviceToHost));
    return TIDE_OK;
  }
  auto f = res->map.find(block);
  if (f != res->map.end()) {
    const int idx = f->second;
    res->cv.wait(lk, [&] { return !res->ent[idx].loading; });
    auto& e = res->ent[idx];
    if (e.valid) {
      res->wait_fence(e);
      std::memcpy(dst, e.buf, res->rec);
      return TIDE_OK;
    }
  }
  lk.unlock();
  if (res->store.odirect) {
    char* al = res->alloc_host(res->rec);
    tide_status r = res->store.read(block, al);
    std::memcpy(dst, al, res->rec);
    res->free_host(al);
    return r;
  }
  return res->store.read(block, dst);
}

tide_status tide_tier_get_stats(const tide_residency* res, tide_tier_stats* out) {
  TIDE_CHECK_ARG(res && out, "null argument");
  *out = res->st;
  return TIDE_OK;
}

tide_status tide_tier_spheres(const tide_residency* res, float* out, int64_t n_blocks) {
  TIDE_CHECK_ARG(res && out && n_blocks == res->K, "bad arguments");
  std::memcpy(out, res->h_spheres.data(), 16 * res->K);
  return TIDE_OK;
}

tide_status tide_tier_resident(const tide_residency* res, int32_t* out, int64_t cap, int32_t* n) {
  TIDE_CHECK_ARG(res && n && (out || cap == 0) && cap >= 0, "bad arguments");
  std::lock_guard<std::mutex> g(const_cast<tide_residency*>(res)->mu);
  *n = (int32_t)res->R.size();
  if ((int64_t)res->R.size() > cap) {
    set_error("resident set of %zu blocks exceeds cap %lld", res->R.size(), (long long)cap);
    return TIDE_ECAPACITY;
  }
  std::copy(res->R.begin(), res->R.end(), out);
  return TIDE_OK;
}

}  // extern "C"

void tide::residency_shape(const tide_residency* res, int64_t* n_rows, int32_t* block_rows) {
  *n_rows = res->N;
  *block_rows = res->B;
}
