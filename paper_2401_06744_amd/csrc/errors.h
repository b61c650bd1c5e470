// Error reporting of the C ABI: entry points run their body through
// `guarded`, which turns a thrown Fail into its inpaint_status and keeps the
// message for inpaint_last_error() on the calling thread.  Host-only.
#pragma once

#include <new>
#include <string>

#include "inpaint.h"

namespace inpaint {

extern thread_local std::string g_err;

struct Fail {
  int code;
};

// Record msg for the calling thread and throw Fail{code}.
[[noreturn]] void fail(int code, const std::string& msg);

template <class Fn>
int guarded(Fn&& fn) {
  g_err.clear();
  try {
    return fn();
  } catch (const Fail& e) {
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return INPAINT_E_NOMEM;
  } catch (...) {
    g_err = "unexpected exception";
    return INPAINT_E_DEVICE;
  }
}

}  // namespace inpaint
