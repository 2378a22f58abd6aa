// Shared host-side helpers of the HIP library: error propagation to the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <new>
#include <string>

#include "nacrith.h"

namespace nc {

struct Error {
  nc_status status;
  std::string msg;
};

void set_last_error(const std::string& msg);

[[noreturn]] inline void fail(nc_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  throw Error{st, std::string(buf)};
}

#define NC_HIP(call)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      ::nc::fail(e_ == hipErrorOutOfMemory ? NC_E_NOMEM : NC_E_DEVICE, "%s: %s (%s:%d)", \
                 #call, hipGetErrorString(e_), __FILE__, __LINE__);                     \
  } while (0)

#define NC_CHECK(cond, st, ...)            \
  do {                                     \
    if (!(cond)) ::nc::fail(st, __VA_ARGS__); \
  } while (0)

// Runs f() and converts any exception into an nc_status plus a thread-local message.
template <class F>
nc_status guard(F&& f) {
  try {
    f();
    set_last_error("");
    return NC_OK;
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.status;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return NC_E_NOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return NC_E_STATE;
  } catch (...) {
    set_last_error("unknown error");
    return NC_E_STATE;
  }
}

inline size_t ceil_div(size_t a, size_t b) { return (a + b - 1) / b; }

}  // namespace nc
