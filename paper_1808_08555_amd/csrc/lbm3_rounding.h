// Storage of FP64 results in FP32 with deterministic stochastic rounding: the helpers
// shared by the two- and three-dimensional steps.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

namespace tcg {
namespace {

// 32-bit integer mixer ("lowbias32", from Wellons' hash-prospector search): a bijection with
// low output bias; it seeds the per-node sequence of the stochastic rounding (NodeBits).
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
// the smallest normal float (2^-126; zero stays zero) the conversion rounds to nearest.
// Beyond the float range the conversion gives +-Inf (+-FLT_MAX within half an ulp of it), so
// overflow still shows.  Inf stays Inf (its low bits are zero, so nothing carries), and so
// does a NaN here: every NaN a step of FP32 storage meets comes from float inputs or from
// the arithmetic, whose NaNs are the quiet NaN or carry an input's payload, so its 29 low
// mantissa bits are zero as well.  No range test per value (it cost 14% of the FP32-storage
// step at 4096^2).
__device__ __forceinline__ float round_stochastic(double v, uint32_t bits)
{
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint64_t s = (u + (uint64_t)(bits >> 3)) & ~((1ull << 29) - 1ull);
    return (float)__longlong_as_double((long long)s);
}

// Random bits for the stochastic rounding of the values one node stores in one step: a
// lowbias32 hash of the node's key (step salt, node index) seeds a Weyl sequence (Weyl's
// equidistribution theorem: x_q = x_0 + q d mod 2^32 with d = 2^32 (sqrt(5) - 1)/2), one
// 32-bit value per stored value, in store order, one add each.  The hash makes x_0, so
// every x_q, uniform and independent from node to node and step to step, which is what
// the rounding's unbiasedness needs; within a node the values are tied to one another
// (each rounding is still unbiased on its own).  An xorshift32 step per value instead cost
// 7% of the FP32-storage step at 4096^2.
struct NodeBits {
    uint32_t x;
    __device__ explicit NodeBits(uint32_t key) : x(mix32(key)) {}
    __device__ uint32_t next()
    {
        x += 0x9e3779b9u;
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
