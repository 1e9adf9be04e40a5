// Error reporting shared by every C entry point: status codes out, text in a thread-local
// buffer read by tanq_last_error(); no exception crosses the ABI.
#pragma once

#include <new>
#include <string>

#include "internal.hpp"

namespace tanq {

tanq_status set_last_error(tanq_status code, const std::string& msg);
void clear_last_error();

template <typename F>
tanq_status guarded(F&& f) {
  try {
    clear_last_error();
    f();
    return TANQ_OK;
  } catch (const Error& e) {
    return set_last_error(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return set_last_error(TANQ_E_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return set_last_error(TANQ_E_STATE, e.what());
  } catch (...) {
    return set_last_error(TANQ_E_STATE, "unknown failure");
  }
}

}  // namespace tanq
