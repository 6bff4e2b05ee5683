// Internal helpers shared by the library's translation units.
#pragma once

#include <cstdarg>
#include <cstdint>

#include "hfr.h"

// Records a message for hfr_last_error() and returns `code`.
hfr_status hfr_fail(hfr_status code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
// Clears the last error message (a successful call leaves "").
hfr_status hfr_ok();

#define HFR_REQUIRE(cond, ...)                          \
    do {                                                \
        if (!(cond)) return hfr_fail(HFR_EINVAL, __VA_ARGS__); \
    } while (0)

inline bool hfr_is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

inline int hfr_log2i(int64_t v)
{
    int l = 0;
    while ((int64_t(1) << l) < v) ++l;
    return l;
}
