// Host-side helpers shared by the library's translation units: the thread-local error
// state behind mickey_last_error(), launch checking and the launch-failure injection of
// mickey_debug_fail_launch().
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "../../include/mickey.h"

namespace mickey_host {

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int ok();
int check_launch(const char *what);
// Prefixes the current error message with `prefix: ` (the code is kept).
void prefix_error(const char *prefix);
// Called before a kernel launch or an asynchronous copy that changes a state: reports
// MICKEY_EDEVICE without making the launch when an injected failure falls due, else
// MICKEY_OK.
int launch_guard(const char *what);

inline size_t pad64(size_t n) { return (n + 63) / 64 * 64; }

}  // namespace mickey_host
