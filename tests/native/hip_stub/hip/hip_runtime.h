// Host-only stand-in for the two HIP runtime calls the batch scheduler makes,
// so that the scheduler compiles with g++ under the sanitizers (no GPU).
#pragma once
#include <cstddef>

typedef int hipError_t;
enum { hipSuccess = 0 };

inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipMemGetInfo(size_t* free_bytes, size_t* total_bytes) {
    *free_bytes = (size_t)8 << 30;
    *total_bytes = (size_t)16 << 30;
    return hipSuccess;
}
