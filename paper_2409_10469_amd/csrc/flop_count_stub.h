// host stand-in for counting arithmetic of the device step (not a GPU build)
#pragma once
#include <cmath>
#include <cstdint>
#include <cstring>
#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __shared__
#define __launch_bounds__(x)
inline uint32_t __umulhi(uint32_t a, uint32_t b) { return (uint32_t)(((uint64_t)a * b) >> 32); }
inline float __int_as_float(int i) { float f; std::memcpy(&f, &i, 4); return f; }
inline int __float_as_int(float f) { int i; std::memcpy(&i, &f, 4); return i; }
inline int __double2loint(double d) { int64_t i; std::memcpy(&i, &d, 8); return (int)(i & 0xffffffff); }
inline int __double2hiint(double d) { int64_t i; std::memcpy(&i, &d, 8); return (int)(i >> 32); }
inline double __hiloint2double(int hi, int lo) { int64_t i = ((int64_t)hi << 32) | (uint32_t)lo; double d; std::memcpy(&d, &i, 8); return d; }
inline int __builtin_amdgcn_update_dpp(int, int v, int, int, int, bool) { return v; }
inline float __expf(float x) { return expf(x); }
inline void sincospif(float x, float* s, float* c) { *s = sinf(M_PI * x); *c = cosf(M_PI * x); }
inline void sincospi(double x, double* s, double* c) { *s = sin(M_PI * x); *c = cos(M_PI * x); }
using std::min; using std::max;
typedef int hipError_t;
typedef void* hipStream_t;
