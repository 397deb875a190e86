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
// needs no event.
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

void release_cached_locked(Pool& P) {
  for (auto& kv : P.free_blocks)
    for (void* b : kv.second) (void)hipFree(b);
  P.free_blocks.clear();
  P.cached_bytes = 0;
}

}  // namespace

hipError_t pool_alloc(void** out, size_t bytes) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const size_t cls = size_class(bytes);
  Pool& P = pool();
  std::lock_guard<std::mutex> g(P.mu);
  auto it = P.free_blocks.find({dev, cls});
  if (it != P.free_blocks.end() && !it->second.empty()) {
    *out = it->second.back();
    it->second.pop_back();
    P.cached_bytes -= cls;
  } else {
    e = hipMalloc(out, cls);
    if (e == hipErrorOutOfMemory) {
      (void)hipGetLastError();
      release_cached_locked(P);
      e = hipMalloc(out, cls);
    }
    if (e != hipSuccess) {
      *out = nullptr;
      return e;
    }
  }
  P.live[*out] = {dev, cls};
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
  P.live.erase(it);
}

}  // namespace ss
