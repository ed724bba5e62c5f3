// vit_guard.h -- host allocation failures at the C ABI.
//
// Entry points that allocate run their bodies under guard_entry(), so that no
// C++ exception leaves the C ABI: a failed host allocation (std::bad_alloc from
// the library's containers, or a failed checkpoint) returns VIT_ENOMEM, and so
// does any other standard-library exception (thread or synchronisation
// resources), with its message.  alloc_checkpoint() marks the library's host
// allocation points; vit_debug_fail_allocations(n) makes the next n of them
// fail, for tests of the error paths.
#pragma once

#include <exception>
#include <new>

#include "vit.h"
#include "vit_internal.h"

namespace vit {

// True (and one fewer pending failure) when a failure was requested.
bool alloc_checkpoint_fails();

inline void alloc_checkpoint() {
  if (alloc_checkpoint_fails()) throw std::bad_alloc();
}

template <class F>
int guard_entry(const char *name, F &&body) noexcept {
  try {
    return body();
  } catch (const std::bad_alloc &) {
    return api_fail(VIT_ENOMEM, "%s: host allocation failed", name);
  } catch (const std::exception &e) {
    return api_fail(VIT_ENOMEM, "%s: %s", name, e.what());
  } catch (...) {
    return api_fail(VIT_ENOMEM, "%s: host resource failure", name);
  }
}

}  // namespace vit
