// Host-side helpers shared by the library's C-ABI sources (not public).
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <exception>
#include <new>
#include <string>
#include <vector>

#include "ugks_internal.h"

namespace ugks {
namespace host {

struct HipFail {
  hipError_t e;
  const char* what;
};

#define HIP_TRY(call)                              \
  do {                                             \
    hipError_t _e = (call);                        \
    if (_e != hipSuccess) throw HipFail{_e, #call}; \
  } while (0)

// A roctx range over one library call, shown by rocprofv3 --marker-trace.
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

struct InvalidArg {
  std::string msg;
};

template <typename T>
inline T* dalloc(ugks_ctx* c, size_t n) {
  if (n == 0) n = 1;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, n * sizeof(T));
  if (e != hipSuccess) throw HipFail{e, "hipMalloc"};
  c->allocations.push_back(p);
  c->bytes += (int64_t)(n * sizeof(T));
  return static_cast<T*>(p);
}

template <typename T>
inline T* upload(ugks_ctx* c, const std::vector<T>& v) {
  T* p = dalloc<T>(c, v.size());
  if (!v.empty()) HIP_TRY(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return p;
}


inline void fail_if(bool cond, const std::string& msg) {
  if (cond) throw InvalidArg{msg};
}

// The remaining handlers of a C-ABI entry point, after its HipFail handler:
// no exception crosses the ABI.  ERR(obj, code, msg) records the message
// and returns the code.
#define UGKS_CATCH_REST(ERR, OBJ)                                                   \
  catch (const ::ugks::host::InvalidArg& e_) {                                     \
    return ERR(OBJ, UGKS_EINVAL, e_.msg);                                           \
  }                                                                                 \
  catch (const std::bad_alloc&) {                                                   \
    return ERR(OBJ, UGKS_ENOMEM, "host memory allocation failed");                  \
  }                                                                                 \
  catch (const std::exception& e_) {                                                \
    return ERR(OBJ, UGKS_EHIP, std::string("internal error: ") + e_.what());        \
  }                                                                                 \
  catch (...) {                                                                     \
    return ERR(OBJ, UGKS_EHIP, "internal error");                                   \
  }

}  // namespace host
}  // namespace ugks
