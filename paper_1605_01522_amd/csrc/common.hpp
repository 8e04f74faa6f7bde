// Shared host-side definitions of the gfx950 n-field solver library:
// error handling, owned device buffers and the device CSR type.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "nfield.h"

namespace nf {

struct NfError : std::runtime_error {
  int code;
  NfError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define NF_HIP(call)                                                                         \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      throw ::nf::NfError(NFIELD_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define NF_CHECK(cond, code, msg)                        \
  do {                                                  \
    if (!(cond)) throw ::nf::NfError((code), (msg));    \
  } while (0)

// Per-context cache of device blocks.  Buffers created while a context's
// pool is installed (g_pool, set by every entry point for the call) come from
// and return to that pool instead of hipMalloc / hipFree (hipFree waits for
// the whole device).  Blocks are kept by size class; a block freed during a
// call is reused only by later work of the same context, and a call on a
// different stream than the previous one first waits for that stream, so a
// reused block is never still in use by an earlier kernel.
struct DevPool {
  size_t live = 0;                 // bytes in buffers handed out
  size_t cached = 0;               // bytes held for reuse
  hipStream_t last = nullptr;
  bool used = false;
  std::multimap<size_t, void*> blocks;
  static size_t size_class(size_t b) {
    if (b <= 4096) return (b + 255) & ~(size_t)255;
    const int lg = 63 - __builtin_clzll((unsigned long long)b);
    const size_t g = (size_t)1 << (lg - 3);
    return (b + g - 1) & ~(g - 1);
  }
  void* get(size_t cls) {
    auto it = blocks.find(cls);
    if (it != blocks.end()) {
      void* p = it->second;
      blocks.erase(it);
      cached -= cls;
      live += cls;
      return p;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, cls);
    if (e != hipSuccess && !blocks.empty()) {          // give the cache back and retry once
      (void)hipGetLastError();
      trim();
      e = hipMalloc(&p, cls);
    }
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    live += cls;
    return p;
  }
  void put(void* p, size_t cls) {
    blocks.emplace(cls, p);
    live -= cls;
    cached += cls;
  }
  // give a block back to the device instead of the cache (hipFree waits for
  // the device)
  void drop(void* p, size_t cls) {
    live -= cls;
    (void)hipFree(p);
  }
  void trim() {
    if (blocks.empty()) return;
    (void)hipDeviceSynchronize();
    for (auto& b : blocks) (void)hipFree(b.second);
    blocks.clear();
    cached = 0;
  }
  void enter(hipStream_t s) {
    if (used && s != last) (void)hipStreamSynchronize(last);
    used = true;
    last = s;
  }
  ~DevPool() { trim(); }
};
extern thread_local DevPool* g_pool;

// Owned device buffer (move-only).
template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DevPool* pool = nullptr;
  size_t cls = 0;
  DBuf() = default;
  explicit DBuf(size_t n_) { alloc(n_); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n), pool(o.pool), cls(o.cls) { o.p = nullptr; o.n = 0; o.pool = nullptr; o.cls = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p; n = o.n; pool = o.pool; cls = o.cls;
      o.p = nullptr; o.n = 0; o.pool = nullptr; o.cls = 0;
    }
    return *this;
  }
  ~DBuf() { release(); }
  void alloc(size_t n_) {
    release();
    n = n_;
    if (n) {
      if (g_pool) {
        pool = g_pool;
        cls = DevPool::size_class(n * sizeof(T));
        p = (T*)pool->get(cls);
      } else {
        if (hipMalloc((void**)&p, n * sizeof(T)) != hipSuccess) {
          (void)hipGetLastError();
          p = nullptr;
        }
      }
      if (!p) {
        pool = nullptr;
        n = 0;
        throw NfError(NFIELD_ENOMEM, "device allocation of " + std::to_string(n_ * sizeof(T)) + " bytes failed");
      }
    }
  }
  void release() {
    if (p) {
      if (pool) pool->put(p, cls);
      else (void)hipFree(p);
    }
    p = nullptr;
    n = 0;
    pool = nullptr;
    cls = 0;
  }
  // release to the device, not to the context's cache (the caller makes
  // sure no queued work still uses the buffer)
  void free_now() {
    if (p) {
      if (pool) pool->drop(p, cls);
      else (void)hipFree(p);
    }
    p = nullptr;
    n = 0;
    pool = nullptr;
    cls = 0;
  }
  T* get() const { return p; }
  size_t bytes() const { return n * sizeof(T); }
};

// Device CSR, 32-bit indices (sizes are checked to fit), FP64 values and an
// optional FP32 copy for the reduced-precision hierarchy.
struct DCsr {
  int nr = 0, nc = 0;
  int64_t nnz = 0;
  DBuf<int> ptr, col;
  DBuf<double> val;
  DBuf<float> val32;
  // block copy of a matrix made of dense bsr_b x bsr_b node blocks (built by
  // the Gauss-Seidel set-up of its level; read by that smoother and by SpMVs
  // with one right-hand side outside the set-up): bsr_ptr / bsr_col the
  // block rows and column nodes; node u's values start at bsr_ptr[u] b^2,
  // entry by entry (entry (q, c) of its blocks in order at offset
  // (q b + c) times its block count, then the next)
  int bsr_b = 0;
  int64_t bsr_nblk = 0;
  DBuf<int> bsr_ptr, bsr_col;
  DBuf<double> bsr_val;
  DBuf<float> bsr_val32;
  void bsr_release() {
    bsr_b = 0;
    bsr_nblk = 0;
    bsr_ptr.release();
    bsr_col.release();
    bsr_val.release();
    bsr_val32.release();
  }
  bool empty() const { return nnz == 0 && ptr.p == nullptr; }
};

// Host copy of a device CSR (tests / inspection).
struct HCsr {
  int nr = 0, nc = 0;
  std::vector<int> ptr, col;
  std::vector<double> val;
};

}  // namespace nf
