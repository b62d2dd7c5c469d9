// Host-side helpers shared by the library's translation units: the thread-local error
// state behind mickey_last_error() and launch checking.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "../../include/mickey.h"

namespace mickey_host {

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int ok();
int check_launch(const char *what);
// Saves the current error, runs `cleanup`, then restores the error with a prefix.
void prefix_error(const char *prefix);

inline size_t pad64(size_t n) { return (n + 63) / 64 * 64; }

}  // namespace mickey_host
