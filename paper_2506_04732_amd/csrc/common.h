// Shared helpers of libt2s2: error state, HIP checks, complex arithmetic.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdio>
#include <stdexcept>
#include <string>

namespace t2s2 {

// Kernel classes timed by the optional event instrumentation.
enum KernelClass {
  KC_GEMM = 0, KC_GEMM_C, KC_TTMV, KC_SCHUR, KC_HESS, KC_JACOBI, KC_CHOL, KC_TRTRI, KC_TREVEC, KC_KRONSOLVE,
  KC_HESSSOLVE, KC_OTHER, KC_COUNT
};

// When enabled, every instrumented launch is bracketed by two HIP events on
// its stream; algorithmic bytes / flops of the launch are accumulated.
void timing_record_begin(hipStream_t s, int cls, double bytes, double flops);
void timing_record_end(hipStream_t s);
bool timing_enabled(int cls = -1);  // cls < 0: any class

struct TimedScope {
  hipStream_t s;
  bool on;
  TimedScope(hipStream_t s_, int cls, double bytes, double flops, bool enable = true)
      : s(s_), on(enable && timing_enabled(cls)) {
    if (on) timing_record_begin(s, cls, bytes, flops);
  }
  ~TimedScope() {
    if (on) timing_record_end(s);
  }
};

// Error carried from deep inside the library to the C ABI boundary.
struct Error : public std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);

}  // namespace t2s2

#define T2S2_HIP(call)                                                              \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess)                                                           \
      throw ::t2s2::Error(4, std::string(#call) + ": " + hipGetErrorString(e_) +    \
                                 " (" + __FILE__ + ":" + std::to_string(__LINE__) + ")"); \
  } while (0)

#define T2S2_CHECK(cond, msg)                                        \
  do {                                                               \
    if (!(cond)) throw ::t2s2::Error(1, std::string(msg));           \
  } while (0)

#define T2S2_LAUNCH_CHECK() T2S2_HIP(hipGetLastError())

// ---- complex double as double2 ------------------------------------------
__host__ __device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline double2 cmulc(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__host__ __device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__host__ __device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ inline double cabs(double2 a) { return hypot(a.x, a.y); }
__device__ inline double2 cdiv(double2 a, double2 b) {
  // Smith's algorithm
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y / b.x, den = b.x + b.y * r;
    return make_double2((a.x + a.y * r) / den, (a.y - a.x * r) / den);
  }
  const double r = b.x / b.y, den = b.x * r + b.y;
  return make_double2((a.x * r + a.y) / den, (a.y * r - a.x) / den);
}
// ---- complex single as float2 (the FP32 factorisations of mixed precision)
__host__ __device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__host__ __device__ inline float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__host__ __device__ inline float cabs2(float2 a) { return a.x * a.x + a.y * a.y; }
__device__ inline float cabs(float2 a) { return hypotf(a.x, a.y); }
__device__ inline float2 cdiv(float2 a, float2 b) {
  if (fabsf(b.x) >= fabsf(b.y)) {
    const float r = b.y / b.x, den = b.x + b.y * r;
    return make_float2((a.x + a.y * r) / den, (a.y - a.x * r) / den);
  }
  const float r = b.x / b.y, den = b.x * r + b.y;
  return make_float2((a.x * r + a.y) / den, (a.y * r - a.x) / den);
}

// complex type of a real type, and its constructor
template <class R> struct CxOf;
template <> struct CxOf<double> {
  using type = double2;
  __host__ __device__ static double2 make(double re, double im) { return make_double2(re, im); }
};
template <> struct CxOf<float> {
  using type = float2;
  __host__ __device__ static float2 make(float re, float im) { return make_float2(re, im); }
};

__device__ inline double2 csqrt(double2 z) {
  const double r = hypot(z.x, z.y);
  if (r == 0.0) return make_double2(0.0, 0.0);
  double t = sqrt(0.5 * (r + fabs(z.x)));
  if (z.x >= 0.0) return make_double2(t, z.y / (2.0 * t));
  return make_double2(fabs(z.y) / (2.0 * t), z.y >= 0.0 ? t : -t);
}
