// Shared device/host helpers for the Gaussian-state -> MPS library (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define GBS_K_MAX 12          // max distinct occupied modes per kept state (2^k <= chi <= 4096)
#define GBS_CHI_MAX 4096
#define GBS_CHI_MAX_SITE 16384  // single-site builds (no truncation sweep)

// Device-side error codes written into the handle's error word.
enum {
  GBS_DEVERR_NONE = 0,
  GBS_DEVERR_NOT_PD = 1,       // a Cholesky pivot was not positive
  GBS_DEVERR_NOT_PURE = 2,     // purity residual above tolerance
  GBS_DEVERR_WILLIAMSON = 3,   // symplectic pairing failed
  GBS_DEVERR_SINGULAR = 4,     // U not invertible (cannot happen for valid input)
  GBS_DEVERR_HASH = 5,         // kept-set index lookup failed
  GBS_DEVERR_KMAX = 6,         // too many occupied modes in a kept state
  GBS_DEVERR_JACOBI = 7,       // Jacobi of a Williamson form did not converge
  GBS_DEVERR_JACOBI_BOND = 8,  // Hermitian Jacobi of a bond environment did not converge
  GBS_DEVERR_ALIGN = 9,        // the two sides of a cut counted different entangled pairs
};

struct cplx64 { double re, im; };
struct cplx32 { float re, im; };

template <typename T> struct cplx_of;
template <> struct cplx_of<double> { typedef cplx64 type; };
template <> struct cplx_of<float> { typedef cplx32 type; };

template <typename C> struct real_of;
template <> struct real_of<cplx64> { typedef double type; };
template <> struct real_of<cplx32> { typedef float type; };

template <typename C> __host__ __device__ inline C cmake(typename real_of<C>::type r, typename real_of<C>::type i) { C c; c.re = r; c.im = i; return c; }
template <typename C> __host__ __device__ inline C cadd(C a, C b) { return cmake<C>(a.re + b.re, a.im + b.im); }
template <typename C> __host__ __device__ inline C csub(C a, C b) { return cmake<C>(a.re - b.re, a.im - b.im); }
template <typename C> __host__ __device__ inline C cmul(C a, C b) { return cmake<C>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); }
template <typename C> __host__ __device__ inline C cconj(C a) { return cmake<C>(a.re, -a.im); }
template <typename C> __host__ __device__ inline C cscale(C a, typename real_of<C>::type s) { return cmake<C>(a.re * s, a.im * s); }
template <typename C> __host__ __device__ inline typename real_of<C>::type cabs2(C a) { return a.re * a.re + a.im * a.im; }
// a += b * c
template <typename C> __host__ __device__ inline void cfma(C& a, C b, C c) {
  a.re += b.re * c.re - b.im * c.im;
  a.im += b.re * c.im + b.im * c.re;
}

// Atomically record the first device error.
__device__ inline void gbs_set_error(int* err, int code) { atomicCAS(err, 0, code); }

// ---------------------------------------------------------------------------
// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter-based RNG.
struct philox4 { uint32_t v[4]; };
__host__ __device__ inline philox4 philox4x32_10(philox4 ctr, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)M0 * ctr.v[0];
    uint64_t p1 = (uint64_t)M1 * ctr.v[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    philox4 n;
    n.v[0] = hi1 ^ ctr.v[1] ^ k0;
    n.v[1] = lo1;
    n.v[2] = hi0 ^ ctr.v[3] ^ k1;
    n.v[3] = lo0;
    ctr = n;
    k0 += W0;
    k1 += W1;
  }
  return ctr;
}
// Uniform in [0,1) with 24 random bits.
__host__ __device__ inline float u01_24(uint32_t x) { return (float)(x >> 8) * (1.0f / 16777216.0f); }

// splitmix64 (Steele, Lea, Flood 2014) for the additive state hash.
__host__ __device__ inline uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

#define HIP_CHECK_RET(...)                                         \
  do {                                                             \
    hipError_t _e = (__VA_ARGS__);                                 \
    if (_e != hipSuccess) return set_hip_error(_e, #__VA_ARGS__);  \
  } while (0)
