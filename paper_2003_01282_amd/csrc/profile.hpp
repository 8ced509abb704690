// Stage timing hooks (see profile.hip).  prof_begin returns -1 when profiling
// is off, so the launch path costs one relaxed atomic load.
#pragma once

#include <hip/hip_runtime.h>

namespace slaq {
int prof_begin(const char* name, hipStream_t st);
void prof_end(int token, hipStream_t st);
}  // namespace slaq

#define SLAQ_TIMED(NAME, STREAM, ...)                        \
    do {                                                     \
        const int tok_ = ::slaq::prof_begin(NAME, STREAM);   \
        __VA_ARGS__;                                         \
        ::slaq::prof_end(tok_, STREAM);                      \
    } while (0)
