// Process-wide caching pool of device memory for libhelm.
//
// Every device buffer of the library (a handle's coefficients and factors, the sweep's slab
// iterates and exchange slots, the FGMRES bases) comes from here.  A freed block stays
// cached, keyed by size, and is handed out again to a later request of about its size, so a
// program that repeatedly sets up a handle and solves (an inversion loop, a benchmark) asks
// the HIP runtime for memory once, not per handle and per solve: allocating and returning
// tens of gigabytes through the runtime costs seconds of device time per call.
//
// Stream safety: a block is returned with the stream its last user queued work on; an event
// recorded there at return makes a later user on another stream wait for that work before
// touching the block (a user on the same stream is ordered by the stream itself).
//
// When the runtime cannot satisfy a request, the cached blocks of that device are released
// (after the device has drained) and the request is retried once.  helm_pool_trim releases
// all cached blocks; helm_pool_stats reports the bytes cached and in use.
#include <map>
#include <mutex>
#include <unordered_map>

#include "common.h"

namespace {

struct Block {
  void* p = nullptr;
  size_t bytes = 0;
  int dev = 0;
  hipStream_t stream = nullptr;  // stream of the last user (at return)
  hipEvent_t done = nullptr;     // recorded on that stream at return (null: nothing pending)
};

struct Pool {
  std::mutex mu;
  std::multimap<std::pair<int, size_t>, Block> cached;  // (device, bytes) -> block
  std::unordered_map<void*, Block> live;
  size_t cached_bytes = 0, live_bytes = 0;
};

// never destroyed: libhelm may be unloaded after the HIP runtime has torn down, and freeing
// device memory or events from a static destructor at that point is undefined
Pool& pool() {
  static Pool* p = new Pool();
  return *p;
}

// sizes are rounded up: 512 B below 1 MiB, 2 MiB above
size_t round_up(size_t bytes) {
  if (bytes == 0) bytes = 1;
  const size_t g = bytes < (1u << 20) ? 512 : (2u << 20);
  return (bytes + g - 1) / g * g;
}

// releases every cached block of device dev (dev < 0: all devices); the caller holds the lock
void release_cached(Pool& P, int dev) {
  for (auto it = P.cached.begin(); it != P.cached.end();) {
    if (dev >= 0 && it->first.first != dev) {
      ++it;
      continue;
    }
    Block& b = it->second;
    if (b.done) {
      (void)hipEventSynchronize(b.done);
      (void)hipEventDestroy(b.done);
    }
    (void)hipFree(b.p);
    P.cached_bytes -= b.bytes;
    it = P.cached.erase(it);
  }
}

}  // namespace

hipError_t pool_alloc(void** out, size_t bytes, hipStream_t s) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const size_t want = round_up(bytes);
  Pool& P = pool();
  std::lock_guard<std::mutex> lock(P.mu);
  // the smallest cached block that holds the request without wasting more than an eighth
  auto it = P.cached.lower_bound({dev, want});
  if (it != P.cached.end() && it->first.first == dev && it->second.bytes <= want + want / 8) {
    Block b = it->second;
    P.cached.erase(it);
    P.cached_bytes -= b.bytes;
    if (b.done) {
      if (b.stream != s) e = hipStreamWaitEvent(s, b.done, 0);
      (void)hipEventDestroy(b.done);
      b.done = nullptr;
      if (e != hipSuccess) {
        (void)hipFree(b.p);
        return e;
      }
    }
    b.stream = s;
    P.live[b.p] = b;
    P.live_bytes += b.bytes;
    *out = b.p;
    return hipSuccess;
  }
  void* p = nullptr;
  e = hipMalloc(&p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    release_cached(P, dev);
    e = hipMalloc(&p, want);
    if (e != hipSuccess) return e;
  }
  Block b;
  b.p = p;
  b.bytes = want;
  b.dev = dev;
  b.stream = s;
  P.live[p] = b;
  P.live_bytes += want;
  *out = p;
  return hipSuccess;
}

void pool_free(void* p, hipStream_t s) {
  if (!p) return;
  Pool& P = pool();
  std::lock_guard<std::mutex> lock(P.mu);
  auto it = P.live.find(p);
  if (it == P.live.end()) return;
  Block b = it->second;
  P.live.erase(it);
  P.live_bytes -= b.bytes;
  b.stream = s;
  b.done = nullptr;
  hipEvent_t ev = nullptr;
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) {
    if (hipEventRecord(ev, s) == hipSuccess) {
      b.done = ev;
    } else {
      (void)hipEventDestroy(ev);
      (void)hipStreamSynchronize(s);   // no event: the block is free once its stream drains
    }
  } else {
    (void)hipStreamSynchronize(s);
  }
  P.cached.insert({{b.dev, b.bytes}, b});
  P.cached_bytes += b.bytes;
}

size_t pool_cached_bytes(int dev) {
  Pool& P = pool();
  std::lock_guard<std::mutex> lock(P.mu);
  size_t acc = 0;
  for (const auto& kv : P.cached)
    if (kv.first.first == dev) acc += kv.second.bytes;
  return acc;
}

hipError_t device_free_bytes(size_t* avail) {
  size_t fr = 0, total = 0;
  hipError_t e = hipMemGetInfo(&fr, &total);
  if (e != hipSuccess) return e;
  int dev = 0;
  e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  *avail = fr + pool_cached_bytes(dev);
  return hipSuccess;
}

extern "C" {

void helm_pool_trim(void) {
  Pool& P = pool();
  std::lock_guard<std::mutex> lock(P.mu);
  release_cached(P, -1);
}

void helm_pool_stats(size_t* cached_bytes, size_t* live_bytes) {
  Pool& P = pool();
  std::lock_guard<std::mutex> lock(P.mu);
  if (cached_bytes) *cached_bytes = P.cached_bytes;
  if (live_bytes) *live_bytes = P.live_bytes;
}

}  // extern "C"
