// Value policies: arithmetic type A, storage type T, and the rounding to
// storage applied at the end of every sweep.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace srj {

struct StF64 {
    using A = double;
    using T = double;
    static constexpr int bytes = 8;
    __device__ static A load(T v) { return v; }
    __device__ static T store(A v) { return v; }
    __device__ static A round(A v) { return v; }
};

struct StF32 {
    using A = float;
    using T = float;
    static constexpr int bytes = 4;
    __device__ static A load(T v) { return v; }
    __device__ static T store(A v) { return v; }
    __device__ static A round(A v) { return v; }
};

struct StF16 {
    using A = float;
    using T = _Float16;
    static constexpr int bytes = 2;
    __device__ static A load(T v) { return static_cast<float>(v); }
    // hardware conversion: round to nearest even, subnormals kept, overflow to inf
    __device__ static T store(A v) { return static_cast<_Float16>(v); }
    __device__ static A round(A v) { return load(store(v)); }
};

struct StBF16 {
    using A = float;
    using T = uint16_t;
    static constexpr int bytes = 2;
    __device__ static A load(T v) { return __uint_as_float(static_cast<uint32_t>(v) << 16); }
    // round to nearest even on the upper 16 bits: add 0x7fff plus the lowest
    // kept bit, then truncate; a carry into the exponent gives the next binade
    // or infinity
    __device__ static T store(A v)
    {
        uint32_t u = __float_as_uint(v);
        if ((u & 0x7f800000u) == 0x7f800000u)  // inf or nan: keep (quiet the nan)
            return static_cast<T>((u >> 16) | ((u & 0x007fffffu) ? 0x40u : 0u));
        u += 0x7fffu + ((u >> 16) & 1u);
        return static_cast<T>(u >> 16);
    }
    __device__ static A round(A v) { return load(store(v)); }
};

}  // namespace srj
