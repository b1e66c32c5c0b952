// Internal declarations of the banded FEAST library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/feastband.h"

namespace fb {

// ------------------------------------------------------------------ complex
// aligned to its full size, so that a complex element moves with one 64-bit
// (complex64) or 128-bit (complex128) LDS access rather than two 32-bit ones
template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T x, y;
};
using c64 = cx<float>;
using c128 = cx<double>;


template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T a, T b) {
  cx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
// Loads and stores of global memory.  Pointers that reach a kernel through
// job tables (or a runtime choice between LDS and global memory) are
// otherwise accessed with flat instructions, which also count against the
// LDS wait counter, so that every LDS wait waits for them too; going through
// a pointer in the global address space gives global loads and stores.
#define FB_GMEM __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ T gld(const T* p) {
  return *(const FB_GMEM T*)p;
}
template <typename T>
__device__ __forceinline__ cx<T> gld(const cx<T>* p) {
  const FB_GMEM T* q = (const FB_GMEM T*)p;
  return mk(q[0], q[1]);
}
template <typename T>
__device__ __forceinline__ void gst(T* p, T v) {
  *(FB_GMEM T*)p = v;
}
template <typename T>
__device__ __forceinline__ void gst(cx<T>* p, cx<T> v) {
  FB_GMEM T* q = (FB_GMEM T*)p;
  q[0] = v.x;
  q[1] = v.y;
}

template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) {
  return mk(a.x + b.x, a.y + b.y);
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) {
  return mk(a.x - b.x, a.y - b.y);
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) {
  return mk(s * a.x, s * a.y);
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> cconj(cx<T> a) {
  return mk(a.x, -a.y);
}
template <typename T>
__host__ __device__ __forceinline__ T cabs2(cx<T> a) {
  return a.x * a.x + a.y * a.y;
}
// acc += a * b
template <typename T>
__host__ __device__ __forceinline__ void cmac(cx<T>& acc, cx<T> a, cx<T> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
// acc += conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ void cmacc(cx<T>& acc, cx<T> a, cx<T> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
}
// 1 / a
template <typename T>
__host__ __device__ __forceinline__ cx<T> cinv(cx<T> a) {
  T d = a.x * a.x + a.y * a.y;
  return mk(a.x / d, -a.y / d);
}
template <typename To, typename Ti>
__host__ __device__ __forceinline__ cx<To> ccast(cx<Ti> a) {
  return mk((To)a.x, (To)a.y);
}

// ------------------------------------------------------------------ errors
#define FB_HIP(expr)                                  \
  do {                                                \
    hipError_t _e = (expr);                           \
    if (_e != hipSuccess) return -1000 - (int)_e;     \
  } while (0)

#define FB_TRY(expr)          \
  do {                        \
    int _r = (expr);          \
    if (_r != 0) return _r;   \
  } while (0)

// ------------------------------------------------------------------ workspace
// Bump allocator over the caller's workspace.  In query mode (base == NULL)
// it only accumulates the size.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
  template <typename T>
  T* take(size_t count) {
    size_t off = (used + 255) & ~(size_t)255;
    used = off + count * sizeof(T);
    if (base == nullptr) return nullptr;
    return reinterpret_cast<T*>(base + off);
  }
  bool fits() const { return base == nullptr || used <= cap; }
};

// ------------------------------------------------------------------ band
// Internal copy of B: diagonal-major, Bd[d*n + j] = B(j+d, j) (complex128,
// zero beyond the matrix), with the norms and Gershgorin bounds.
struct Band {
  int64_t n;
  int b;         // bandwidth used by the kernels (>= 1)
  int b0;        // declared bandwidth (may be 0)
  bool cplx;
  c128* Bd;      // dev, (b+1) * n
  double* stats; // dev, 4: ||B||_1, g_lo, g_hi, count of NaN / Inf entries
  // block-tridiagonal copy with nb x nb blocks (nb = b rounded up to 16):
  // Bblk[(k*3 + s) * nb*nb], s = 0: B(k,k-1), 1: B(k,k), 2: B(k,k+1), column-major
  c128* Bblk;
  int nb;
  int K;
};

// Kernels launched from the host side (defined in the .hip files).
// blocks = false skips the block-tridiagonal copy (only the FP64 residual reads
// it).  Returns FB_ERR_NONFINITE when B holds a NaN or an infinity.
int ingest_band(const fb_band* B, Band& out, Arena& ar, hipStream_t st, bool blocks = true);
int band_stats_host(const Band& bd, double* out3, hipStream_t st);
// FB_ERR_NONFINITE when one of the nblk column-major blocks P[i] (rows x
// cols[i], leading dimension ld[i] in elements; complex128 or double) holds a
// NaN or an infinity.  part_dev: scratch of kFiniteParts doubles per block
// (one int32 counter per block is used).  Synchronises.
int check_finite_blocks(int nblk, const void* const* P, const int64_t* ld, const int32_t* cols,
                        int64_t rows, bool cplx, double* part_dev, hipStream_t st);
constexpr int kFiniteParts = 64;

// inertia for nshift shifts (dev shifts array), counts dev int32 x3
int launch_inertia(const Band& bd, int nshift, const double* shifts_dev,
                   int32_t* cnt_dev, void* scratch, hipStream_t st);
size_t inertia_scratch_bytes(const Band& bd, int nshift);

int device_cus();

}  // namespace fb
