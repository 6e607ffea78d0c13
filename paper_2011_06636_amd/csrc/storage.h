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
    // round to nearest even on the upper 16 bits (a carry into the exponent
    // gives the next binade or infinity): gfx950's conversion instruction,
    // which gives the same bits as adding 0x7fff plus the lowest kept bit and
    // truncating for every finite and infinite binary32 value (checked
    // exhaustively over all 2^32 patterns on the device); a NaN stays a NaN
    __device__ static T store(A v) { return __builtin_bit_cast(T, static_cast<__bf16>(v)); }
    __device__ static A round(A v) { return load(store(v)); }
};

}  // namespace srj
