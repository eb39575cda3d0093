// Shared internals of libnys: error state, storage-type traits, device
// buffers, and launch helpers.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/nys.h"

namespace nys {

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);

#define NYS_CHECK_HIP(expr)                                                  \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess) {                                                  \
      ::nys::set_error("%s:%d %s -> %s", __FILE__, __LINE__, #expr,          \
                       hipGetErrorString(e_));                               \
      return NYS_EHIP;                                                       \
    }                                                                        \
  } while (0)

#define NYS_REQUIRE(cond, ...)                                               \
  do {                                                                       \
    if (!(cond)) {                                                           \
      ::nys::set_error(__VA_ARGS__);                                         \
      return NYS_EINVAL;                                                     \
    }                                                                        \
  } while (0)

#define NYS_TRY(expr)                                                        \
  do {                                                                       \
    nys_status s_ = (expr);                                                  \
    if (s_ != NYS_OK) return s_;                                             \
  } while (0)

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// ---------------------------------------------------------------- bf16
__device__ __host__ inline float bf16_to_f32(uint16_t b) {
  uint32_t u = static_cast<uint32_t>(b) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

__device__ __host__ inline uint16_t f32_to_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu))
    return static_cast<uint16_t>((u >> 16) | 0x40u);          // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);                            // nearest even
  return static_cast<uint16_t>(u >> 16);
}

// Storage type S -> compute type C, with load/store conversions.
template <class S> struct Io;
template <> struct Io<double> {
  using C = double;
  __device__ static double ld(const double* p, size_t i) { return p[i]; }
  __device__ static void st(double* p, size_t i, double v) { p[i] = v; }
};
template <> struct Io<float> {
  using C = float;
  __device__ static float ld(const float* p, size_t i) { return p[i]; }
  __device__ static void st(float* p, size_t i, float v) { p[i] = v; }
};
template <> struct Io<uint16_t> {
  using C = float;
  __device__ static float ld(const uint16_t* p, size_t i) { return bf16_to_f32(p[i]); }
  __device__ static void st(uint16_t* p, size_t i, float v) { p[i] = f32_to_bf16(v); }
};

inline size_t dtype_size(nys_dtype d) {
  return d == NYS_F64 ? 8 : d == NYS_F32 ? 4 : 2;
}

// ---------------------------------------------------------------- buffers
// Caller-owned device scratch of one call, handed out as a stack: take()
// returns the next 256-byte aligned part, Mark restores the top on scope
// exit.  Exhaustion is an argument error (the caller's workspace is smaller
// than the size query returned); nothing is ever allocated.
struct Scratch {
  char* base = nullptr;
  size_t cap = 0, off = 0;
  Scratch() = default;
  Scratch(void* p, size_t n) : base(static_cast<char*>(p)), cap(p ? n : 0) {}
  template <class T> T* take(size_t count) {
    const size_t b = (count * sizeof(T) + 255) / 256 * 256;
    if (off + b > cap) {
      set_error("workspace of %zu bytes is too small (needs more than %zu)", cap, off + b);
      return nullptr;
    }
    T* p = reinterpret_cast<T*>(base + off);
    off += b;
    return p;
  }
  struct Mark {
    Scratch* s;
    size_t off;
    explicit Mark(Scratch* sc) : s(sc), off(sc ? sc->off : 0) {}
    ~Mark() { if (s) s->off = off; }
  };
};

inline constexpr size_t ws_round(size_t b) { return (b + 255) / 256 * 256; }

// ptr = count values of type T from the scratch bound to a handle.
#define NYS_TAKE(scr, T, ptr, count)                                         \
  do {                                                                       \
    if (!(scr)) {                                                            \
      ::nys::set_error("no workspace bound to the handle");                  \
      return NYS_EINVAL;                                                     \
    }                                                                        \
    ptr = (scr)->template take<T>(count);                                    \
    if (!ptr) return NYS_EINVAL;                                             \
  } while (0)

// Device buffer owned by a handle, allocated when the handle is created and
// freed by its destroy call.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  nys_status ensure(size_t want) {
    if (want <= bytes) return NYS_OK;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    if (hipMalloc(&p, want) != hipSuccess) {
      set_error("hipMalloc(%zu) failed", want);
      return NYS_ENOMEM;
    }
    bytes = want;
    return NYS_OK;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

inline unsigned cdiv(int64_t a, int64_t b) { return static_cast<unsigned>((a + b - 1) / b); }

inline nys_status launch_check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("launch of %s failed: %s", what, hipGetErrorString(e));
    return NYS_EHIP;
  }
  return NYS_OK;
}

// ---------------------------------------------------------------- handles
struct OpImpl;  // defined in ops.hip

}  // namespace nys

// Public handle types.
// Filters of the periodised Daubechies-4 wavelet: scaling h and wavelet
// g_k = (-1)^k h_{7-k}, in both precisions (kernel arguments).
struct Db4Coef {
  double hd[8], gd[8];
  float hf[8], gf[8];
};

struct nys_op_s {
  nys_op_desc d{};
  Db4Coef db4{};                  // filled when d.wavelet == NYS_WAVELET_DB4
  int64_t N = 0, M = 0;
  std::vector<double> psf;        // k*k row-major
  // psf[a][b] = sep_u[a] * sep_v[b] when sep != 0 (rank-1 PSF, e.g. Gaussian)
  int sep = 0;
  double sep_u[32] = {}, sep_v[32] = {};
  nys::DevBuf psf_dev;            // [flipped psf f64 | psf f64 | flipped f32 | psf f32]
  nys::DevBuf trig;               // per view: cos, sin (f64) then (f32)
  // the caller's workspace while a call enqueues work (null otherwise):
  // intermediates of composed operators, Daubechies-4 pass scratch, the
  // fan-beam adjoint's accumulation, transposed images of the parallel beam
  nys::Scratch* scr = nullptr;
  // fan beam: per view cos, sin (f64), then per ray (view-major) f0, g and the
  // step-length scale signed + for steps along rows, - along columns (f64);
  // filled at creation when the gathered adjoint applies (fan_gather)
  nys::DevBuf rays;
  bool fan_gather = false;
};

struct nys_pc_s {
  int64_t N = 0, ell = 0;
  int64_t ldu = 0;                // pitch of U's columns (elements), >= N
  int64_t ell_pad = 0;            // rows of U allocated: ell rounded up to 16, zero padded
  int32_t u_dtype = NYS_F32;
  int32_t tail = 0;
  double pinv_norm_cache = -1.0;  // ||P^{-1}|| once read back from the device
  nys::DevBuf U;                  // ell*N
  nys::DevBuf meta;               // FP64 device block, see factor.hip
  nys::DevBuf ssn_ws;             // semismooth Newton state, partials, stored LU factors
                                  // (allocated with the handle)
  // the caller's workspace while a call enqueues work (null otherwise):
  // block partials of U^T v, coefficients
  nys::Scratch* scr = nullptr;
  // pinned, coherent host word (8 seq + outcome bits) written by the
  // semismooth Newton decision kernel and read by the host without a stream
  // synchronisation; the sequence number counts decisions
  unsigned long long* hflag = nullptr;
  unsigned long long flag_seq = 0;
  // warm-start output of the semismooth Newton call being enqueued (may be
  // null): the decision that ends the iteration writes the root there
  double* ssn_gout = nullptr;
  // h of that call: soft threshold (0) or the clip to [lo, hi] (1)
  int ssn_box = 0;
  double ssn_lo = 0.0, ssn_hi = 0.0;
  // the FP32 semismooth Newton workspace holds LU factors of a Jacobian of
  // this preconditioner (cleared whenever the factorisation is redone or the
  // workspace is reallocated)
  bool ssn_lu_valid = false;
  bool ssn_lu_hint = false;   // the last decision read reported stored factors
  // calls being captured into a graph: a fixed sequence of trials whose
  // kernels skip themselves on the device state (no host decision), with
  // ssn_slots Newton-and-trial rounds after the first two trials; the
  // outcome goes to ssn_status[0] (NYS_ENOTFINITE) or [1] (NYS_ENOCONV)
  bool ssn_device = false;
  int ssn_slots = 2;
  int32_t* ssn_status = nullptr;
};

namespace nys {
// A caller's workspace of ws_bytes for a call that needs `need` bytes:
// large enough, non-null when needed, 256-byte aligned.
inline nys_status check_workspace(const void* ws, size_t ws_bytes, size_t need, const char* what) {
  NYS_REQUIRE(ws_bytes >= need, "%s: workspace of %zu bytes < %zu", what, ws_bytes, need);
  NYS_REQUIRE(need == 0 || ws, "%s: null workspace", what);
  NYS_REQUIRE(reinterpret_cast<uintptr_t>(ws) % 256 == 0, "%s: workspace not 256-byte aligned",
              what);
  return NYS_OK;
}

// Binds a caller's workspace to the handles of one call while it enqueues
// work (the previous binding, if any, is restored on exit).
struct WsBind {
  Scratch s;
  nys_op op;
  nys_pc pc;
  Scratch* prev_op = nullptr;
  Scratch* prev_pc = nullptr;
  WsBind(void* ws, size_t bytes, nys_op o, nys_pc p) : s(ws, bytes), op(o), pc(p) {
    if (op) { prev_op = op->scr; op->scr = &s; }
    if (pc) { prev_pc = pc->scr; pc->scr = &s; }
  }
  WsBind(const WsBind&) = delete;
  WsBind& operator=(const WsBind&) = delete;
  ~WsBind() {
    if (op) op->scr = prev_op;
    if (pc) pc->scr = prev_pc;
  }
};
}  // namespace nys
