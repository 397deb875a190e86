// Caching device allocator of the library.
//
// hipMalloc is slow and hipFree synchronises the whole device, which would
// stall every stream that is solving while another thread builds or retires
// a request.  Blocks are therefore rounded to size classes (quarter steps
// between powers of two) and kept on per-device free lists after release;
// they return to the driver only when an allocation fails (then every cached
// block is released and the allocation retried).  A block is released only
// after the work that used it has completed (every release point in the
// library follows a stream synchronisation), so handing it to another stream
// needs no event.  The pool's lock guards its lists only: hipMalloc and
// hipFree run without it, so a thread waiting in the driver (hipFree waits
// for the device) never holds up another thread's cached allocations.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "ss_internal.h"

namespace ss {

namespace {

struct Pool {
  std::mutex mu;
  std::map<std::pair<int, size_t>, std::vector<void*>> free_blocks;   // (device, class) -> blocks
  std::unordered_map<void*, std::pair<int, size_t>> live;             // block -> (device, class)
  size_t cached_bytes = 0;
  size_t live_bytes = 0;
  uint64_t driver_allocs = 0;   // successful allocations from the driver
};

Pool& pool() {
  static Pool* p = new Pool();   // never destroyed: blocks may be released during process teardown
  return *p;
}

size_t size_class(size_t bytes) {
  if (bytes <= 256) return 256;
  size_t p = 1;
  while ((p << 1) <= bytes) p <<= 1;
  const size_t step = p >> 2;
  return (bytes + step - 1) / step * step;
}

// every cached block, taken off the lists (the caller frees them without the lock)
std::vector<void*> take_cached(Pool& P) {
  std::lock_guard<std::mutex> g(P.mu);
  std::vector<void*> out;
  for (auto& kv : P.free_blocks) out.insert(out.end(), kv.second.begin(), kv.second.end());
  P.free_blocks.clear();
  P.cached_bytes = 0;
  return out;
}

}  // namespace

hipError_t pool_alloc(void** out, size_t bytes) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const size_t cls = size_class(bytes);
  Pool& P = pool();
  {
    std::lock_guard<std::mutex> g(P.mu);
    auto it = P.free_blocks.find({dev, cls});
    if (it != P.free_blocks.end() && !it->second.empty()) {
      *out = it->second.back();
      it->second.pop_back();
      P.cached_bytes -= cls;
      P.live_bytes += cls;
      P.live[*out] = {dev, cls};
      return hipSuccess;
    }
  }
  e = hipMalloc(out, cls);
  if (e == hipErrorOutOfMemory) {   // give the cached blocks back to the driver and try again
    (void)hipGetLastError();
    for (void* b : take_cached(P)) (void)hipFree(b);
    e = hipMalloc(out, cls);
  }
  if (e != hipSuccess) {
    *out = nullptr;
    return e;
  }
  std::lock_guard<std::mutex> g(P.mu);
  P.live[*out] = {dev, cls};
  P.live_bytes += cls;
  P.driver_allocs += 1;
  return hipSuccess;
}

void pool_free(void* p) {
  if (!p) return;
  Pool& P = pool();
  std::lock_guard<std::mutex> g(P.mu);
  auto it = P.live.find(p);
  if (it == P.live.end()) return;
  P.free_blocks[it->second].push_back(p);
  P.cached_bytes += it->second.second;
  P.live_bytes -= it->second.second;
  P.live.erase(it);
}

void pool_stats(int64_t* live_bytes, int64_t* cached_bytes, int64_t* driver_allocs) {
  Pool& P = pool();
  std::lock_guard<std::mutex> g(P.mu);
  *live_bytes = (int64_t)P.live_bytes;
  *cached_bytes = (int64_t)P.cached_bytes;
  *driver_allocs = (int64_t)P.driver_allocs;
}

// ---------------------------------------------------------------- pinned result buffers
// Pinned host memory for the small device-to-host result buffers of a solve (per-problem sums and
// states).  hipHostMalloc is slow and hipHostFree waits for the device -- in the batch pipeline
// one part's free stalled behind the other parts' kernels for milliseconds -- so these buffers
// are cached like device blocks: size classes, per-device free lists, never returned to the
// driver (so a small class is allocated in slabs of several blocks).  A buffer is released only after the stream that filled it has been synchronised.

namespace {

constexpr size_t kPinnedSlab = 8;   // blocks per allocation of a small pinned class

Pool& pinned_pool() {
  static Pool* p = new Pool();   // never destroyed, like the device pool
  return *p;
}

}  // namespace

hipError_t pinned_alloc(void** out, size_t bytes) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const size_t cls = size_class(bytes);
  Pool& P = pinned_pool();
  {
    std::lock_guard<std::mutex> g(P.mu);
    auto it = P.free_blocks.find({dev, cls});
    if (it != P.free_blocks.end() && !it->second.empty()) {
      *out = it->second.back();
      it->second.pop_back();
      P.cached_bytes -= cls;
      P.live[*out] = {dev, cls};
      return hipSuccess;
    }
  }
  // a miss takes a slab of several blocks of the class (small classes): concurrent solves then
  // find their buffers cached after the first one, instead of each paying an allocation that
  // also disturbs the work in flight
  const size_t n = cls <= (size_t(64) << 10) ? kPinnedSlab : 1;
  char* slab = nullptr;
  e = hipHostMalloc((void**)&slab, n * cls, hipHostMallocDefault);
  if (e != hipSuccess) {
    *out = nullptr;
    return e;
  }
  std::lock_guard<std::mutex> g(P.mu);
  *out = slab;
  P.live[*out] = {dev, cls};
  for (size_t i = 1; i < n; ++i) {
    P.free_blocks[{dev, cls}].push_back(slab + i * cls);
    P.cached_bytes += cls;
  }
  return hipSuccess;
}

void pinned_free(void* p) {
  if (!p) return;
  Pool& P = pinned_pool();
  std::lock_guard<std::mutex> g(P.mu);
  auto it = P.live.find(p);
  if (it == P.live.end()) return;
  P.free_blocks[it->second].push_back(p);
  P.cached_bytes += it->second.second;
  P.live.erase(it);
}

namespace {

struct ReadbackBuf {   // the calling thread's pinned staging of device-to-host reads
  char* p = nullptr;
  size_t cap = 0;
  ~ReadbackBuf() { pinned_free(p); }   // back to the cache: no device call here
};
thread_local ReadbackBuf t_readback;

}  // namespace

ss_status Readback::add(void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return SS_OK;
  size_t off = (used + 255) & ~size_t(255);
  if (off + bytes > t_readback.cap) {
    if (!parts.empty()) {   // the queued copies target the current buffer
      SS_TRY(sync());
      off = 0;
    }
    pinned_free(t_readback.p);
    t_readback.p = nullptr;
    const size_t cap = std::max({bytes, 2 * t_readback.cap, size_t(64) << 10});
    t_readback.cap = 0;
    const hipError_t e = pinned_alloc((void**)&t_readback.p, cap);
    if (e != hipSuccess) return fail(SS_ENOMEM, std::string("pinned allocation: ") + hipGetErrorString(e));
    t_readback.cap = cap;
  }
  const hipError_t e = hipMemcpyAsync(t_readback.p + off, src, bytes, hipMemcpyDeviceToHost, stream);
  if (e != hipSuccess) return fail(SS_EDEVICE, std::string("device-to-host copy: ") + hipGetErrorString(e));
  parts.push_back(Part{dst, off, bytes});
  used = off + bytes;
  return SS_OK;
}

ss_status Readback::sync() {
  const hipError_t e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return fail(SS_EDEVICE, std::string("stream synchronisation: ") + hipGetErrorString(e));
  for (const Part& q : parts) std::memcpy(q.dst, t_readback.p + q.off, q.bytes);
  parts.clear();
  used = 0;
  return SS_OK;
}

// ---------------------------------------------------------------- pinned staging of uploads
// A copy from pageable host memory is staged by the runtime and holds the calling thread until
// the stream has reached it, which drains the stream before the next launch is even issued.
// Uploads are therefore copied into pinned host memory first; the device copy then only queues.
// A thread takes a ring of pinned chunks from a shared list on its first upload and gives it back
// when it ends (rings live as long as the process, so short-lived threads allocate nothing).  A
// chunk holds the copies of one stream, and its event, recorded behind each of them, covers them
// all; a chunk is refilled only after its event has completed.  Events belong to the device
// current when the chunk was first used.

namespace {

struct PinChunk {
  char* host = nullptr;
  size_t cap = 0, used = 0;
  hipEvent_t ev = nullptr;
  hipStream_t stream = nullptr;
};

constexpr int kPinRing = 3;
constexpr size_t kPinChunk = size_t(4) << 20;

struct PinRing {
  PinChunk chunk[kPinRing];
  int cur = 0;
};

std::mutex g_pin_mu;
std::vector<PinRing*> g_pin_free;

struct PinHolder {
  PinRing* ring = nullptr;
  ~PinHolder() {   // no device calls here: it may run while the process ends
    if (!ring) return;
    std::lock_guard<std::mutex> g(g_pin_mu);
    g_pin_free.push_back(ring);
  }
};

PinRing* pin_ring() {
  thread_local PinHolder holder;
  if (!holder.ring) {
    std::lock_guard<std::mutex> g(g_pin_mu);
    if (!g_pin_free.empty()) {
      holder.ring = g_pin_free.back();
      g_pin_free.pop_back();
    } else {
      holder.ring = new PinRing();   // never destroyed: copies may be in flight at teardown
    }
  }
  return holder.ring;
}

// A slot of `bytes` in the calling thread's pinned ring for a copy queued on `stream`; pin_submit
// queues the copy from it and records the chunk's event behind it.
hipError_t pin_reserve(size_t bytes, hipStream_t stream, PinChunk** out, char** host) {
  PinRing& ring = *pin_ring();
  PinChunk* c = &ring.chunk[ring.cur];
  const size_t need = (bytes + 255) & ~size_t(255);
  if (c->stream != stream || c->used + need > c->cap) {
    if (c->used > 0) {   // move on; the next chunk is refilled once its copies are done
      ring.cur = (ring.cur + 1) % kPinRing;
      c = &ring.chunk[ring.cur];
      if (c->used > 0) {
        const hipError_t e = hipEventSynchronize(c->ev);
        if (e != hipSuccess) return e;
        c->used = 0;
      }
    }
    c->stream = stream;
  }
  if (!c->ev) {
    const hipError_t e = hipEventCreateWithFlags(&c->ev, hipEventDisableTiming);
    if (e != hipSuccess) {
      c->ev = nullptr;
      return e;
    }
  }
  if (need > c->cap) {   // the chunk is empty here
    if (c->host) (void)hipHostFree(c->host);
    c->host = nullptr;
    c->cap = 0;
    const size_t cap = std::max(kPinChunk, need);
    const hipError_t e = hipHostMalloc((void**)&c->host, cap, hipHostMallocDefault);
    if (e != hipSuccess) {
      c->host = nullptr;
      return e;
    }
    c->cap = cap;
  }
  *out = c;
  *host = c->host + c->used;
  return hipSuccess;
}

hipError_t pin_submit(PinChunk* c, void* dst, const char* h, size_t bytes, hipStream_t stream) {
  hipError_t e = hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipEventRecord(c->ev, stream);
  if (e == hipSuccess) c->used += (bytes + 255) & ~size_t(255);
  return e;
}

}  // namespace

hipError_t h2d(void* dst, const void* src, size_t bytes, hipStream_t stream) {
  if (bytes == 0) return hipSuccess;
  PinChunk* c = nullptr;
  char* h = nullptr;
  hipError_t e = pin_reserve(bytes, stream, &c, &h);
  if (e != hipSuccess) return e;
  std::memcpy(h, src, bytes);
  return pin_submit(c, dst, h, bytes, stream);
}

ss_status Upload::commit(void** block, hipStream_t stream) {
  *block = nullptr;
  size_t total = 0;
  std::vector<size_t> off(pieces.size());
  for (size_t i = 0; i < pieces.size(); ++i) {
    off[i] = total;
    total += (pieces[i].bytes + 255) & ~size_t(255);
  }
  hipError_t e = pool_alloc(block, std::max<size_t>(total, 256));
  if (e != hipSuccess) {
    *block = nullptr;
    return fail(e == hipErrorOutOfMemory ? SS_ENOMEM : SS_EDEVICE,
                std::string("device allocation: ") + hipGetErrorString(e));
  }
  char* base = static_cast<char*>(*block);
  for (size_t i = 0; i < pieces.size(); ++i) pieces[i].point(base + off[i]);
  if (total == 0) return SS_OK;
  PinChunk* c = nullptr;
  char* h = nullptr;
  e = pin_reserve(total, stream, &c, &h);
  if (e == hipSuccess) {
    for (size_t i = 0; i < pieces.size(); ++i)
      if (pieces[i].bytes) std::memcpy(h + off[i], pieces[i].host, pieces[i].bytes);
    e = pin_submit(c, base, h, total, stream);
  }
  if (e != hipSuccess) return fail(SS_EDEVICE, std::string("host-to-device copy: ") + hipGetErrorString(e));
  return SS_OK;
}

}  // namespace ss
