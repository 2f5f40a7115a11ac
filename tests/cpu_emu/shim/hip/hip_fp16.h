// CPU build: IEEE half conversions through the host compiler's _Float16 (round to nearest
// even, subnormals kept).
#pragma once
#include <cstring>

struct __half { _Float16 h; };

inline __half __float2half_rn(float f) { return __half{(_Float16)f}; }
inline float __half2float(__half h) { return (float)h.h; }
inline unsigned short __half_as_ushort(__half h) { unsigned short u; std::memcpy(&u, &h.h, 2); return u; }
inline __half __ushort_as_half(unsigned short u) { __half h; std::memcpy(&h.h, &u, 2); return h; }
