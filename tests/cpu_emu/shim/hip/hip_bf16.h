// CPU build: bfloat16 conversions (round to nearest even; NaN kept quiet).
#pragma once
#include <cstring>

struct __hip_bfloat16 { unsigned short b; };

inline __hip_bfloat16 __float2bfloat16(float f) {
  unsigned u;
  std::memcpy(&u, &f, 4);
  __hip_bfloat16 r;
  if ((u & 0x7fffffffu) > 0x7f800000u) {
    r.b = (unsigned short)((u >> 16) | 0x40u);
  } else {
    u += 0x7fffu + ((u >> 16) & 1u);
    r.b = (unsigned short)(u >> 16);
  }
  return r;
}
inline unsigned short __bfloat16_as_ushort(__hip_bfloat16 h) { return h.b; }
