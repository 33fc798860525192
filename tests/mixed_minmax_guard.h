// Included (with -include) only by tests/test_sources_cpu.py.  HIP's math
// headers overload min and max for two arithmetic types of different kinds
// by converting both to double; in index and byte-count arithmetic that puts
// integer work in FP64 vector registers.  A deleted overload for two
// different integral types makes every such call ambiguous, so a device
// source that compiles with this header makes none.
#pragma once
#include <type_traits>
template <typename A, typename B,
          typename std::enable_if<std::is_integral<A>::value && std::is_integral<B>::value &&
                                      !std::is_same<A, B>::value,
                                  int>::type = 0>
__device__ double min(A, B) = delete;
template <typename A, typename B,
          typename std::enable_if<std::is_integral<A>::value && std::is_integral<B>::value &&
                                      !std::is_same<A, B>::value,
                                  int>::type = 0>
__device__ double max(A, B) = delete;
