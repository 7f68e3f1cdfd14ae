// Host compilation of the library's multiple-double arithmetic (md.hpp) for
// CPU tests: the device qualifiers become plain (inline) host functions.
#pragma once
#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
