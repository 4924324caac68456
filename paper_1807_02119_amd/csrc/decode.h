// decode.h -- mixed-radix decoding of spin-group indices, shared by the
// device engine and by host code (the planner's range guard and a CPU test
// compile this same header).
//
// A tensor of the network G_T (Sec. III of arXiv:1807.02119) is indexed by
// spins taking q values each.  A contraction step addresses a group of r of
// them by one index 0 <= idx < q^r (first spin most significant); its offset
// in the operand is sum_j digit_j * stride_j.  The digits are peeled off by
// exact division by q with a multiply-high instead of an integer divide.
#pragma once
#include <stdint.h>

#ifdef __HIPCC__
#define KN_HD __host__ __device__
#else
#define KN_HD
#endif

namespace kn {

// Every index QDiv::div accepts: 0 <= x <= kDecodeMax (all non-negative int32).
constexpr int64_t kDecodeMax = 2147483647;

// Exact floor(x / q) for 2 <= q <= 8 and 0 <= x < 2^31.
//
// With l = ceil(log2 q) and m = floor(2^(31+l) / q) + 1 (m < 2^32), write
// m q = 2^(31+l) + d with 1 <= d <= q <= 2^l.  Then
//   x m / 2^(31+l) = x / q + x d / (q 2^(31+l)),
// and the second term is below 2^31 2^l / (q 2^(31+l)) = 1/q, while the
// fractional part of x / q is at most (q-1)/q: the floor is that of x / q.
// The product is formed as the high 32 bits of a 32 x 32-bit product
// (one multiply-high on the GPU), then shifted right by l - 1.
struct QDiv {
  uint32_t m;
  int32_t sh;
  int32_t q;
  KN_HD explicit QDiv(int32_t q_) : m(0), sh(0), q(q_) {
    int32_t l = 0;
    while ((1 << l) < q_) ++l;
    m = (uint32_t)(((uint64_t)1 << (31 + l)) / (uint64_t)q_ + 1);
    sh = l - 1;
  }
  KN_HD inline int32_t div(int32_t x) const {
    const uint32_t hi = (uint32_t)(((uint64_t)(uint32_t)x * (uint64_t)m) >> 32);
    return (int32_t)(hi >> sh);
  }
};

// Offset of value `idx` of a spin group (r spins, strides str[], first spin
// most significant) in its operand.
KN_HD inline int32_t group_off(int32_t idx, const int32_t* str, int32_t r, const QDiv& D) {
  int32_t off = 0;
  for (int32_t j = r - 1; j >= 0; --j) {
    const int32_t qd = D.div(idx);
    off += (idx - qd * D.q) * str[j];
    idx = qd;
  }
  return off;
}

}  // namespace kn
