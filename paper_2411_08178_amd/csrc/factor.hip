// Shifted Nystrom factorisation (Alg. 1 steps 3-8) and the preconditioner of
// eq. (6): Gram of [Omega Y], ell x ell FP64 algebra on one workgroup,
// U = Y_nu R in one pass, and P^{-1} / P applications.

#include <cmath>

#include "common.hpp"
#include "internal.hpp"

namespace nys {

// ================================================================ Gram
// G = Z^T Z for Z = [Omega | Y] (N x 2 ell, column-major).  Each block
// accumulates one 64 x 64 tile (upper triangle of tiles only) over a chunk
// of rows in the compute type C, then writes it in FP64; a second kernel sums
// the chunk partials in FP64 in a fixed order.
constexpr int kGT = 64, kGK = 32;

template <class S, class C>
__global__ __launch_bounds__(256) void gram_partial_kernel(
    const S* __restrict__ omega, const S* __restrict__ Y, int64_t N, int ell, int64_t chunk,
    int ntiles, double* __restrict__ part) {
  // map blockIdx.y to an upper-triangular tile pair (ti <= tj)
  int t = blockIdx.y, ti = 0;
  while (t >= ntiles - ti) { t -= ntiles - ti; ++ti; }
  const int tj = ti + t;
  const int m = 2 * ell;
  const int64_t n0 = static_cast<int64_t>(blockIdx.x) * chunk;
  const int64_t n1 = (n0 + chunk < N) ? n0 + chunk : N;
  __shared__ C As[kGK][kGT + 1];
  __shared__ C Bs[kGK][kGT + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  C acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0;
  for (int64_t nb = n0; nb < n1; nb += kGK) {
    for (int e = threadIdx.x; e < kGK * kGT; e += 256) {
      int col = e / kGK, kk = e - col * kGK;
      int64_t n = nb + kk;
      int ca = ti * kGT + col, cb = tj * kGT + col;
      C va = 0, vb = 0;
      if (n < n1) {
        if (ca < m) va = ca < ell ? Io<S>::ld(omega, static_cast<size_t>(ca) * N + n)
                                  : Io<S>::ld(Y, static_cast<size_t>(ca - ell) * N + n);
        if (cb < m) vb = cb < ell ? Io<S>::ld(omega, static_cast<size_t>(cb) * N + n)
                                  : Io<S>::ld(Y, static_cast<size_t>(cb - ell) * N + n);
      }
      As[kk][col] = va;
      Bs[kk][col] = vb;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < kGK; ++kk) {
      C a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = As[kk][ty * 4 + q];
        b[q] = Bs[kk][tx * 4 + q];
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] += a[p] * b[q];
    }
    __syncthreads();
  }
  const int ntri = ntiles * (ntiles + 1) / 2;
  double* dst = part + (static_cast<size_t>(blockIdx.x) * ntri + blockIdx.y) * kGT * kGT;
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      dst[(ty * 4 + p) * kGT + tx * 4 + q] = static_cast<double>(acc[p][q]);
}

__global__ void gram_reduce_kernel(const double* __restrict__ part, int nchunks, int ntiles,
                                   int ell, double* __restrict__ G) {
  const int ntri = ntiles * (ntiles + 1) / 2;
  const int m = 2 * ell;
  const int64_t total = static_cast<int64_t>(ntri) * kGT * kGT;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int tri = static_cast<int>(e / (kGT * kGT));
    int r = static_cast<int>(e % (kGT * kGT));
    int i = r / kGT, j = r - i * kGT;
    int t = tri, ti = 0;
    while (t >= ntiles - ti) { t -= ntiles - ti; ++ti; }
    int tj = ti + t;
    int gi = ti * kGT + i, gj = tj * kGT + j;
    if (gi >= m || gj >= m) continue;
    double s = 0;
    for (int c = 0; c < nchunks; ++c) s += part[(static_cast<size_t>(c) * ntri + tri) * kGT * kGT + r];
    G[gi * m + gj] = s;
    G[gj * m + gi] = s;
  }
}

// ================================================================ FP64 factor
// One workgroup.  G is the 2 ell x 2 ell Gram: OO = G[0:l, 0:l],
// OY = G[0:l, l:2l], YY = G[l:2l, l:2l].  Work buffers are l x l FP64 each.
struct FactorWork {
  double *Gs, *Cc, *Mv, *X, *M, *V, *R, *ev;
};

__device__ void block_jacobi_eig(double* M, double* V, int L, double* ev, int max_sweeps) {
  // cyclic Jacobi with round-robin (tournament) ordering: each round rotates
  // m/2 disjoint index pairs in parallel.
  __shared__ double rc[64], rs[64];
  __shared__ int rp[64], rq[64];
  __shared__ double red[256];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int m = (L + 1) & ~1;   // even number of slots; slot >= L is a dummy
  for (int e = tid; e < L * L; e += nt) V[e] = (e / L == e % L) ? 1.0 : 0.0;
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    // off-diagonal and total Frobenius norms
    double off = 0, tot = 0;
    for (int e = tid; e < L * L; e += nt) {
      double v = M[e] * M[e];
      tot += v;
      if (e / L != e % L) off += v;
    }
    red[tid] = off;
    __syncthreads();
    for (int s = nt / 2; s > 0; s >>= 1) {
      if (tid < s) red[tid] += red[tid + s];
      __syncthreads();
    }
    double offs = red[0];
    __syncthreads();
    red[tid] = tot;
    __syncthreads();
    for (int s = nt / 2; s > 0; s >>= 1) {
      if (tid < s) red[tid] += red[tid + s];
      __syncthreads();
    }
    double tots = red[0];
    __syncthreads();
    if (offs <= 1e-32 * tots || tots == 0.0) break;
    for (int r = 0; r < m - 1; ++r) {
      const int npairs = m / 2;
      for (int p = tid; p < npairs; p += nt) {
        int a = (p == 0) ? 0 : ((p - 1 + r) % (m - 1)) + 1;
        int bq = m - 1 - p;
        int b = ((bq - 1 + r) % (m - 1)) + 1;
        int i = a < b ? a : b, j = a < b ? b : a;
        double c = 1.0, s = 0.0;
        if (j < L) {
          double apq = M[i * L + j];
          if (apq != 0.0) {
            double tau = (M[j * L + j] - M[i * L + i]) / (2.0 * apq);
            double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        rc[p] = c; rs[p] = s; rp[p] = i; rq[p] = j;
      }
      __syncthreads();
      // rows: M <- J^T M
      for (int e = tid; e < npairs * L; e += nt) {
        int p = e / L, col = e - p * L;
        int i = rp[p], j = rq[p];
        if (j >= L || rs[p] == 0.0) continue;
        double c = rc[p], s = rs[p];
        double mi = M[i * L + col], mj = M[j * L + col];
        M[i * L + col] = c * mi - s * mj;
        M[j * L + col] = s * mi + c * mj;
      }
      __syncthreads();
      // columns: M <- M J, V <- V J
      for (int e = tid; e < npairs * L; e += nt) {
        int p = e / L, row = e - p * L;
        int i = rp[p], j = rq[p];
        if (j >= L || rs[p] == 0.0) continue;
        double c = rc[p], s = rs[p];
        double mi = M[row * L + i], mj = M[row * L + j];
        M[row * L + i] = c * mi - s * mj;
        M[row * L + j] = s * mi + c * mj;
        double vi = V[row * L + i], vj = V[row * L + j];
        V[row * L + i] = c * vi - s * vj;
        V[row * L + j] = s * vi + c * vj;
      }
      __syncthreads();
    }
  }
  for (int e = tid; e < L; e += nt) ev[e] = M[e * L + e];
  __syncthreads();
}

__global__ __launch_bounds__(256) void factor_kernel(const double* __restrict__ G, int L,
                                                     int64_t N, int nu_mode, int tail,
                                                     double mu_in, int max_esc, FactorWork w,
                                                     double* __restrict__ meta) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int m = 2 * L;
  __shared__ double sh_nu, sh_diag;
  __shared__ int sh_fail;
  __shared__ int order[PcMeta::kMaxEll];
  const double eps = 2.220446049250313e-16;
  // ---- shift nu
  if (nu_mode == 0) {
    for (int e = tid; e < L * L; e += nt) w.M[e] = G[(L + e / L) * m + L + e % L];
    __syncthreads();
    block_jacobi_eig(w.M, w.V, L, w.ev, 40);
    if (tid == 0) {
      double mx = 0;
      for (int i = 0; i < L; ++i) mx = fmax(mx, w.ev[i]);
      sh_nu = sqrt(static_cast<double>(N)) * eps * sqrt(fmax(mx, 0.0));
    }
  } else if (tid == 0) {
    double tr = 0;
    for (int i = 0; i < L; ++i) tr += G[i * m + i];
    sh_nu = eps * sqrt(tr);
  }
  __syncthreads();
  double nu = sh_nu;
  // ---- shifted Cholesky with escalation
  int esc = 0;
  for (;; ++esc) {
    for (int e = tid; e < L * L; e += nt) {
      int i = e / L, j = e - i * L;
      double oy = 0.5 * (G[i * m + L + j] + G[j * m + L + i]);
      double oo = 0.5 * (G[i * m + j] + G[j * m + i]);
      w.Gs[e] = oy + nu * oo;
      w.Cc[e] = 0.0;
    }
    if (tid == 0) sh_fail = 0;
    __syncthreads();
    for (int j = 0; j < L; ++j) {
      if (tid == 0) {
        double d = w.Gs[j * L + j];
        for (int k = 0; k < j; ++k) d -= w.Cc[j * L + k] * w.Cc[j * L + k];
        if (!(d > 0.0) || !isfinite(d)) { sh_fail = 1; d = 1.0; }
        sh_diag = sqrt(d);
        w.Cc[j * L + j] = sh_diag;
      }
      __syncthreads();
      if (sh_fail) break;
      double djj = sh_diag;
      for (int i = j + 1 + tid; i < L; i += nt) {
        double s = w.Gs[i * L + j];
        for (int k = 0; k < j; ++k) s -= w.Cc[i * L + k] * w.Cc[j * L + k];
        w.Cc[i * L + j] = s / djj;
      }
      __syncthreads();
    }
    __syncthreads();
    if (!sh_fail) break;
    if (esc >= max_esc) break;
    nu *= 10.0;
    __syncthreads();
  }
  if (sh_fail) {
    if (tid == 0) {
      meta[PcMeta::kStatus] = NYS_ENOTPD;
      meta[PcMeta::kNu] = nu;
      meta[PcMeta::kKeff] = 0;
      meta[PcMeta::kEscal] = esc;
      for (int i = 0; i < L; ++i) { meta[PcMeta::kShat + i] = 0; meta[PcMeta::kD + i] = 0; meta[PcMeta::kE + i] = 0; }
    }
    for (int e = tid; e < L * L; e += nt) w.R[e] = 0.0;
    return;
  }
  // ---- Mv = Y_nu^T Y_nu = YY + nu (OY + OY^T) + nu^2 OO
  for (int e = tid; e < L * L; e += nt) {
    int i = e / L, j = e - i * L;
    w.Mv[e] = G[(L + i) * m + L + j] + nu * (G[i * m + L + j] + G[j * m + L + i]) +
              nu * nu * G[i * m + j];
  }
  __syncthreads();
  // ---- X = C^{-1} Mv (column j per thread), then M = C^{-1} X^T
  for (int j = tid; j < L; j += nt)
    for (int i = 0; i < L; ++i) {
      double s = w.Mv[i * L + j];
      for (int k = 0; k < i; ++k) s -= w.Cc[i * L + k] * w.X[k * L + j];
      w.X[i * L + j] = s / w.Cc[i * L + i];
    }
  __syncthreads();
  for (int j = tid; j < L; j += nt)
    for (int i = 0; i < L; ++i) {
      double s = w.X[j * L + i];                       // (X^T)[i][j]
      for (int k = 0; k < i; ++k) s -= w.Cc[i * L + k] * w.M[k * L + j];
      w.M[i * L + j] = s / w.Cc[i * L + i];
    }
  __syncthreads();
  for (int e = tid; e < L * L; e += nt) {
    int i = e / L, j = e - i * L;
    if (i < j) {
      double a = 0.5 * (w.M[i * L + j] + w.M[j * L + i]);
      w.M[i * L + j] = a;
      w.M[j * L + i] = a;
    }
  }
  __syncthreads();
  // ---- eigen-decomposition M = V diag(S^2) V^T, descending order
  block_jacobi_eig(w.M, w.V, L, w.ev, 60);
  if (tid == 0) {
    for (int i = 0; i < L; ++i) order[i] = i;
    for (int i = 0; i < L; ++i) {           // selection sort, descending
      int best = i;
      for (int k = i + 1; k < L; ++k)
        if (w.ev[order[k]] > w.ev[order[best]]) best = k;
      int t = order[i]; order[i] = order[best]; order[best] = t;
    }
  }
  __syncthreads();
  // ---- R = C^{-T} V S^{-1} (column k per thread, back substitution)
  for (int k = tid; k < L; k += nt) {
    int src = order[k];
    double s2 = w.ev[src];
    double inv = s2 > 0 ? 1.0 / sqrt(s2) : 0.0;
    for (int i = L - 1; i >= 0; --i) {
      double s = w.V[i * L + src];
      for (int q = i + 1; q < L; ++q) s -= w.Cc[q * L + i] * w.R[q * L + k];
      w.R[i * L + k] = s / w.Cc[i * L + i];
    }
    for (int i = 0; i < L; ++i) w.R[i * L + k] *= inv;
  }
  __syncthreads();
  // ---- spectrum and preconditioner coefficients
  if (tid == 0) {
    int keff = 0;
    for (int k = 0; k < L; ++k) {
      double sh = fmax(0.0, w.ev[order[k]] - nu);
      meta[PcMeta::kShat + k] = sh;
      if (sh > 0) keff = k + 1;
    }
    double sK = keff > 0 ? meta[PcMeta::kShat + keff - 1] : 0.0;
    double st = tail == 0 ? sqrt(sK) : sK;
    double mu = mu_in < 0 ? nu : mu_in;
    double pn = 1.0;
    for (int k = 0; k < L; ++k) {
      double sh = meta[PcMeta::kShat + k];
      if (k < keff && sh > 0) {
        meta[PcMeta::kD + k] = (st + mu) / (sh + mu) - 1.0;
        meta[PcMeta::kE + k] = (sh + mu) / (st + mu) - 1.0;
        pn = fmax(pn, (st + mu) / (sh + mu));
      } else {
        meta[PcMeta::kD + k] = 0.0;
        meta[PcMeta::kE + k] = 0.0;
      }
    }
    meta[PcMeta::kNu] = nu;
    meta[PcMeta::kSK] = st;
    meta[PcMeta::kMu] = mu;
    meta[PcMeta::kPinvNorm] = pn;
    meta[PcMeta::kKeff] = keff;
    meta[PcMeta::kEscal] = esc;
    bool finite = isfinite(nu) && isfinite(pn);
    meta[PcMeta::kStatus] = finite ? NYS_OK : NYS_ENOTFINITE;
  }
}

// ================================================================ U
// U[k][n] = sum_j (Y[j][n] + nu Omega[j][n]) R[j][k]; KC outputs per thread.
constexpr int kUK = 32;

template <class S, class T, class C>
__global__ __launch_bounds__(256) void form_u_kernel(const S* __restrict__ omega,
                                                     const S* __restrict__ Y,
                                                     const double* __restrict__ R,
                                                     const double* __restrict__ meta, int64_t N,
                                                     int L, T* __restrict__ U) {
  __shared__ C Rs[PcMeta::kMaxEll][kUK];
  const int k0 = blockIdx.y * kUK;
  for (int e = threadIdx.x; e < L * kUK; e += blockDim.x) {
    int j = e / kUK, kk = e - j * kUK;
    Rs[j][kk] = (k0 + kk < L) ? static_cast<C>(R[j * L + k0 + kk]) : C(0);
  }
  __syncthreads();
  const C nu = static_cast<C>(meta[PcMeta::kNu]);
  const int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (n >= N) return;
  C acc[kUK];
#pragma unroll
  for (int kk = 0; kk < kUK; ++kk) acc[kk] = 0;
  for (int j = 0; j < L; ++j) {
    C z = Io<S>::ld(Y, static_cast<size_t>(j) * N + n) + nu * Io<S>::ld(omega, static_cast<size_t>(j) * N + n);
#pragma unroll
    for (int kk = 0; kk < kUK; ++kk) acc[kk] += z * Rs[j][kk];
  }
#pragma unroll
  for (int kk = 0; kk < kUK; ++kk)
    if (k0 + kk < L) U[static_cast<size_t>(k0 + kk) * N + n] = static_cast<T>(acc[kk]);
}

// ================================================================ apply
// c = U^T v per column (partials over row chunks), coef . c, out = v + U (coef . c)
constexpr int kAK = 32, kAChunk = 1024;

template <class T>
__global__ __launch_bounds__(256) void utv_partial_kernel(const T* __restrict__ U,
                                                          const T* __restrict__ v, int64_t N,
                                                          int L, int nchunks,
                                                          double* __restrict__ part) {
  const int k0 = blockIdx.y * kAK;
  const int col = blockIdx.z;
  const T* vc = v + static_cast<size_t>(col) * N;
  const int64_t n0 = static_cast<int64_t>(blockIdx.x) * kAChunk;
  T acc[kAK];
#pragma unroll
  for (int kk = 0; kk < kAK; ++kk) acc[kk] = 0;
  for (int64_t n = n0 + threadIdx.x; n < n0 + kAChunk && n < N; n += 256) {
    T x = vc[n];
#pragma unroll
    for (int kk = 0; kk < kAK; ++kk)
      if (k0 + kk < L) acc[kk] += U[static_cast<size_t>(k0 + kk) * N + n] * x;
  }
  __shared__ double red[4][kAK];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int kk = 0; kk < kAK; ++kk) {
    double s = static_cast<double>(acc[kk]);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) red[wv][kk] = s;
  }
  __syncthreads();
  if (threadIdx.x < kAK && k0 + threadIdx.x < L) {
    double s = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
    part[(static_cast<size_t>(col) * nchunks + blockIdx.x) * L + k0 + threadIdx.x] = s;
  }
}

__global__ void coef_reduce_kernel(const double* __restrict__ part, int nchunks, int L,
                                   const double* __restrict__ coef, double* __restrict__ cd) {
  const int col = blockIdx.x;
  for (int k = threadIdx.x; k < L; k += blockDim.x) {
    double s = 0;
    for (int c = 0; c < nchunks; ++c) s += part[(static_cast<size_t>(col) * nchunks + c) * L + k];
    cd[static_cast<size_t>(col) * L + k] = coef[k] * s;
  }
}

template <class T>
__global__ __launch_bounds__(256) void u_update_kernel(const T* __restrict__ U,
                                                       const T* __restrict__ v,
                                                       const double* __restrict__ cd, int64_t N,
                                                       int L, T* __restrict__ out) {
  __shared__ T cs[PcMeta::kMaxEll];
  const int col = blockIdx.y;
  for (int k = threadIdx.x; k < L; k += blockDim.x) cs[k] = static_cast<T>(cd[static_cast<size_t>(col) * L + k]);
  __syncthreads();
  const int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (n >= N) return;
  T acc = v[static_cast<size_t>(col) * N + n];
  for (int k = 0; k < L; ++k) acc += U[static_cast<size_t>(k) * N + n] * cs[k];
  out[static_cast<size_t>(col) * N + n] = acc;
}

template <class T>
nys_status pc_coeffs(nys_pc pc, bool inverse, const T* v, int64_t ncols, double* cd,
                     hipStream_t st) {
  const int64_t N = pc->N;
  const int L = static_cast<int>(pc->ell);
  const int nchunks = static_cast<int>(cdiv(N, kAChunk));
  NYS_TRY(pc->work.ensure(sizeof(double) * static_cast<size_t>(ncols) * nchunks * L));
  double* part = pc->work.as<double>();
  hipLaunchKernelGGL((utv_partial_kernel<T>), dim3(nchunks, cdiv(L, kAK), ncols), dim3(256), 0, st,
                     pc->U.as<T>(), v, N, L, nchunks, part);
  NYS_TRY(launch_check("utv_partial_kernel"));
  const double* coef = pc->meta.as<double>() + (inverse ? PcMeta::kD : PcMeta::kE);
  hipLaunchKernelGGL(coef_reduce_kernel, dim3(ncols), dim3(128), 0, st, part, nchunks, L, coef, cd);
  return launch_check("coef_reduce_kernel");
}

template nys_status pc_coeffs<double>(nys_pc, bool, const double*, int64_t, double*, hipStream_t);
template nys_status pc_coeffs<float>(nys_pc, bool, const float*, int64_t, double*, hipStream_t);

template <class T>
nys_status pc_apply(nys_pc pc, bool inverse, const T* v, T* out, int64_t ncols, hipStream_t st) {
  const int64_t N = pc->N;
  const int L = static_cast<int>(pc->ell);
  NYS_TRY(pc->work2.ensure(sizeof(double) * static_cast<size_t>(ncols) * L));
  double* cd = pc->work2.as<double>();
  NYS_TRY(pc_coeffs<T>(pc, inverse, v, ncols, cd, st));
  hipLaunchKernelGGL((u_update_kernel<T>), dim3(cdiv(N, 256), ncols), dim3(256), 0, st,
                     pc->U.as<T>(), v, cd, N, L, out);
  return launch_check("u_update_kernel");
}

template nys_status pc_apply<double>(nys_pc, bool, const double*, double*, int64_t, hipStream_t);
template nys_status pc_apply<float>(nys_pc, bool, const float*, float*, int64_t, hipStream_t);

template <class S>
static nys_status factor_impl(const S* omega, const S* Y, int64_t N, int L,
                              const nys_factor_opts& o, nys_pc pc, hipStream_t st) {
  const int m = 2 * L;
  const int ntiles = static_cast<int>(cdiv(m, kGT));
  const int ntri = ntiles * (ntiles + 1) / 2;
  int64_t nchunks = N / 4096;
  if (nchunks < 1) nchunks = 1;
  if (nchunks > 256) nchunks = 256;
  int64_t chunk = (N + nchunks - 1) / nchunks;
  chunk = (chunk + kGK - 1) / kGK * kGK;
  nchunks = (N + chunk - 1) / chunk;
  size_t part_d = static_cast<size_t>(nchunks) * ntri * kGT * kGT;
  size_t G_d = static_cast<size_t>(m) * m;
  size_t w_d = 7 * static_cast<size_t>(L) * L + L;
  NYS_TRY(pc->work.ensure(sizeof(double) * (part_d + G_d + w_d)));
  double* part = pc->work.as<double>();
  double* G = part + part_d;
  double* wb = G + G_d;
  FactorWork w;
  size_t LL = static_cast<size_t>(L) * L;
  w.Gs = wb; w.Cc = wb + LL; w.Mv = wb + 2 * LL; w.X = wb + 3 * LL; w.M = wb + 4 * LL;
  w.V = wb + 5 * LL; w.R = wb + 6 * LL; w.ev = wb + 7 * LL;
  using C = typename Io<S>::C;
  hipLaunchKernelGGL((gram_partial_kernel<S, C>), dim3(static_cast<unsigned>(nchunks), ntri),
                     dim3(256), 0, st, omega, Y, N, L, chunk, ntiles, part);
  NYS_TRY(launch_check("gram_partial_kernel"));
  hipLaunchKernelGGL(gram_reduce_kernel, dim3(64), dim3(256), 0, st, part,
                     static_cast<int>(nchunks), ntiles, L, G);
  NYS_TRY(launch_check("gram_reduce_kernel"));
  hipLaunchKernelGGL(factor_kernel, dim3(1), dim3(256), 0, st, G, L, N, o.nu_mode, o.tail, o.mu,
                     o.max_escalations < 0 ? 6 : o.max_escalations, w, pc->meta.as<double>());
  NYS_TRY(launch_check("factor_kernel"));
  dim3 ug(cdiv(N, 256), cdiv(L, kUK));
  if (pc->u_dtype == NYS_F64) {
    hipLaunchKernelGGL((form_u_kernel<S, double, double>), ug, dim3(256), 0, st, omega, Y, w.R,
                       pc->meta.as<double>(), N, L, pc->U.as<double>());
  } else {
    hipLaunchKernelGGL((form_u_kernel<S, float, C>), ug, dim3(256), 0, st, omega, Y, w.R,
                       pc->meta.as<double>(), N, L, pc->U.as<float>());
  }
  return launch_check("form_u_kernel");
}

}  // namespace nys

using namespace nys;

extern "C" nys_status nys_factor(const void* omega, const void* Y, nys_dtype in_dt, int64_t N,
                                 int64_t ell, const nys_factor_opts* opts, nys_pc* out,
                                 void* stream) {
  NYS_REQUIRE(omega && Y && out && N > 0, "nys_factor: bad argument");
  NYS_REQUIRE(ell >= 1 && ell <= PcMeta::kMaxEll, "nys_factor: ell must be in [1, %d]", PcMeta::kMaxEll);
  NYS_REQUIRE(ell <= N, "nys_factor: ell > N");
  nys_factor_opts o{0, 0, -1.0, 6, NYS_F32};
  if (opts) o = *opts;
  NYS_REQUIRE(o.u_dtype == NYS_F64 || o.u_dtype == NYS_F32, "nys_factor: u_dtype must be F64/F32");
  NYS_REQUIRE(o.nu_mode == 0 || o.nu_mode == 1, "nys_factor: nu_mode must be 0 or 1");
  NYS_REQUIRE(o.tail == 0 || o.tail == 1, "nys_factor: tail must be 0 or 1");
  auto* pc = new nys_pc_s();
  pc->N = N;
  pc->ell = ell;
  pc->u_dtype = o.u_dtype;
  pc->tail = o.tail;
  nys_status s = pc->U.ensure(dtype_size(static_cast<nys_dtype>(o.u_dtype)) * N * ell);
  if (s == NYS_OK) s = pc->meta.ensure(sizeof(double) * PcMeta::kTotal);
  if (s == NYS_OK) {
    hipStream_t st = as_stream(stream);
    switch (in_dt) {
      case NYS_F64:
        s = factor_impl<double>(static_cast<const double*>(omega), static_cast<const double*>(Y), N,
                                static_cast<int>(ell), o, pc, st);
        break;
      case NYS_F32:
        s = factor_impl<float>(static_cast<const float*>(omega), static_cast<const float*>(Y), N,
                               static_cast<int>(ell), o, pc, st);
        break;
      case NYS_BF16:
        s = factor_impl<uint16_t>(static_cast<const uint16_t*>(omega),
                                  static_cast<const uint16_t*>(Y), N, static_cast<int>(ell), o, pc, st);
        break;
      default:
        set_error("nys_factor: bad dtype");
        s = NYS_EINVAL;
    }
  }
  if (s != NYS_OK) {
    nys_pc_destroy(pc);
    return s;
  }
  *out = pc;
  return NYS_OK;
}

extern "C" void nys_pc_destroy(nys_pc pc) {
  if (!pc) return;
  // the factorisation may still be running on its stream
  (void)hipDeviceSynchronize();
  pc->U.release();
  pc->meta.release();
  pc->work.release();
  pc->work2.release();
  delete pc;
}

extern "C" nys_status nys_pc_info(nys_pc pc, double* shat, double* nu, int32_t* k_eff,
                                  int32_t* status, void* stream) {
  NYS_REQUIRE(pc, "nys_pc_info: null pc");
  std::vector<double> meta(PcMeta::kTotal);
  NYS_CHECK_HIP(hipStreamSynchronize(as_stream(stream)));
  NYS_CHECK_HIP(hipMemcpy(meta.data(), pc->meta.p, sizeof(double) * PcMeta::kTotal,
                          hipMemcpyDeviceToHost));
  if (shat)
    for (int k = 0; k < pc->ell; ++k) shat[k] = meta[PcMeta::kShat + k];
  if (nu) *nu = meta[PcMeta::kNu];
  if (k_eff) *k_eff = static_cast<int32_t>(meta[PcMeta::kKeff]);
  if (status) *status = static_cast<int32_t>(meta[PcMeta::kStatus]);
  return NYS_OK;
}

extern "C" nys_status nys_pc_u(nys_pc pc, const void** u, int64_t* N, int64_t* ell,
                               int32_t* u_dtype) {
  NYS_REQUIRE(pc, "nys_pc_u: null pc");
  if (u) *u = pc->U.p;
  if (N) *N = pc->N;
  if (ell) *ell = pc->ell;
  if (u_dtype) *u_dtype = pc->u_dtype;
  return NYS_OK;
}

extern "C" nys_status nys_pc_copy_u(nys_pc pc, void* dst, void* stream) {
  NYS_REQUIRE(pc && dst, "nys_pc_copy_u: bad argument");
  NYS_CHECK_HIP(hipMemcpyAsync(dst, pc->U.p,
                               dtype_size(static_cast<nys_dtype>(pc->u_dtype)) * pc->N * pc->ell,
                               hipMemcpyDeviceToDevice, as_stream(stream)));
  return NYS_OK;
}

extern "C" nys_status nys_apply(nys_pc pc, int32_t inverse, nys_dtype dt, const void* v, void* out,
                                int64_t ncols, void* stream) {
  NYS_REQUIRE(pc && v && out && ncols > 0 && ncols <= 65535, "nys_apply: bad argument");
  NYS_REQUIRE(static_cast<int32_t>(dt) == pc->u_dtype, "nys_apply: dtype must equal the pc's u_dtype");
  hipStream_t st = as_stream(stream);
  if (dt == NYS_F64)
    return pc_apply<double>(pc, inverse != 0, static_cast<const double*>(v), static_cast<double*>(out),
                            ncols, st);
  return pc_apply<float>(pc, inverse != 0, static_cast<const float*>(v), static_cast<float*>(out),
                         ncols, st);
}
