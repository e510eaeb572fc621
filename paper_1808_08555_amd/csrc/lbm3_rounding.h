// Storage of FP64 results in FP32 with deterministic stochastic rounding: the helpers
// shared by the two- and three-dimensional steps.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

namespace tcg {
namespace {

// 32-bit integer mixer ("lowbias32", from Wellons' hash-prospector search): a bijection with
// low output bias; it seeds the per-node generator of the stochastic rounding (NodeBits).
__device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

// FP64 -> FP32 with stochastic rounding: v lies between two adjacent floats a (toward zero)
// and b (away from zero); the result is b with probability (v - a)/(b - a), else a, so its
// expected value is v.  Round to nearest would lose the sub-ulp per-step changes of the
// near-uniform bulk with a sign that is the same at many nodes, which shows up as a steady
// drift of each fluid's mass.
// In the bits of the double, a is v with the 29 mantissa bits that FP32 lacks cleared (the
// sign is separate, so this is toward zero, in v's own binade); adding a uniform 29-bit r to
// those bits first carries into the kept bits, giving b, exactly when r >= 2^29 - low bits,
// that is with probability (v - a)/(b - a).  The sum then converts to float exactly.  Below
// the smallest normal float (2^-126; zero stays zero) the conversion rounds to nearest;
// beyond the float range and for NaN the result is that of round to nearest, so overflow
// still shows as Inf and a NaN stays a NaN.
__device__ __forceinline__ float round_stochastic(double v, uint32_t bits)
{
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint64_t s = (u + (uint64_t)(bits >> 3)) & ~((1ull << 29) - 1ull);
    const float r = (float)__longlong_as_double((long long)s);
    return fabs(v) <= 3.4028234663852886e38 ? r : (float)v;
}

// Random bits for the stochastic rounding of the values one node stores in one step: a
// lowbias32 hash of the node's key (step salt, node index) seeds Marsaglia's xorshift32
// (shifts 13, 17, 5), which gives one 32-bit output per stored value, in store order.  The
// hash decorrelates neighbouring nodes and steps; the xorshift steps are shifts and xors at
// the full issue rate, where a hash per value would cost two 32-bit integer multiplies,
// which issue at a quarter of the rate.  (xorshift32 must not start at 0, hence the | 1.)
struct NodeBits {
    uint32_t x;
    __device__ explicit NodeBits(uint32_t key) : x(mix32(key) | 1u) {}
    __device__ uint32_t next()
    {
        x ^= x << 13;
        x ^= x >> 17;
        x ^= x << 5;
        return x;
    }
};

// Whether stores round (FP32 storage of FP64 arithmetic).
template <typename S, typename C>
constexpr bool kRounds = sizeof(S) < sizeof(C);

// Store of one value in the storage type S from the compute type C (FP32 storage of FP64
// arithmetic: stochastic rounding with the node's next random bits).
template <typename S, typename C>
__device__ __forceinline__ S to_storage(C v, NodeBits& bits)
{
    if constexpr (kRounds<S, C>)
        return round_stochastic(v, bits.next());
    else
        return S(v);
}

}  // namespace
}  // namespace tcg
