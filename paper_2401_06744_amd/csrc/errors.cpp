// Error reporting of the C ABI (see errors.h).  Host-only.
#include "errors.h"

namespace inpaint {

thread_local std::string g_err;

[[noreturn]] void fail(int code, const std::string& msg) {
  g_err = msg;
  throw Fail{code};
}

}  // namespace inpaint
