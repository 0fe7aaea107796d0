// Error reporting shared by the library's entry points.
#pragma once

// Stores a printf-style detail for lbm_last_error() and returns code.
int lbm_fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
