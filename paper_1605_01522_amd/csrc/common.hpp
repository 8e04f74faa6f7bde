// Shared host-side definitions of the gfx950 n-field solver library:
// error handling, owned device buffers and the device CSR type.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
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

// Device bytes currently owned through DBuf objects created while a counter
// is installed (one counter per context; setup installs it).
extern thread_local size_t* g_acct;

// Owned device buffer (move-only).
template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  size_t* acct = nullptr;
  DBuf() = default;
  explicit DBuf(size_t n_) { alloc(n_); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n), acct(o.acct) { o.p = nullptr; o.n = 0; o.acct = nullptr; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; acct = o.acct; o.p = nullptr; o.n = 0; o.acct = nullptr; }
    return *this;
  }
  ~DBuf() { release(); }
  void alloc(size_t n_) {
    release();
    n = n_;
    if (n) {
      hipError_t e = hipMalloc((void**)&p, n * sizeof(T));
      if (e != hipSuccess) {
        p = nullptr;
        n = 0;
        (void)hipGetLastError();
        throw NfError(NFIELD_ENOMEM, "device allocation of " + std::to_string(n_ * sizeof(T)) + " bytes failed");
      }
      acct = g_acct;
      if (acct) *acct += n * sizeof(T);
    }
  }
  void release() {
    if (p) {
      (void)hipFree(p);
      if (acct) *acct -= n * sizeof(T);
    }
    p = nullptr;
    n = 0;
    acct = nullptr;
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
  bool empty() const { return nnz == 0 && ptr.p == nullptr; }
};

// Host copy of a device CSR (tests / inspection).
struct HCsr {
  int nr = 0, nc = 0;
  std::vector<int> ptr, col;
  std::vector<double> val;
};

}  // namespace nf
