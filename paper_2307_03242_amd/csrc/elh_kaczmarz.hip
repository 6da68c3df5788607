// The paper's coarsest-grid solver (Section 3.2, "Coarsest grid solution";
// parameters in Section 5.3): the pressure is eliminated through its
// diagonal block, and the displacement system
//   S u = b_u - A_up diag(A_pp)^-1 b_p,   S = A_uu - A_up diag(A_pp)^-1 A_pu,
// is solved by FGMRES preconditioned with parallel hybrid Kaczmarz sweeps:
// every sub-region (a box of cells) makes one forward pass of relaxed row
// projections over its own rows on a private copy of the iterate, and each
// unknown then takes the mean of the copies of the sub-regions whose rows
// reach it.  The rows of S are stored per row in a fixed slot pattern (the
// couplings of the operator's stencils); the host builds them once.
//
// Kernels:
//   k_kacz_sweep  one wavefront per (sub-region, rhs): the private copy of
//                 the sub-region's neighbourhood lives in LDS; rows are taken
//                 in ascending global order; lanes hold the row's slots, one
//                 butterfly sum gives a_i . x and every lane applies its
//                 slots' share of the projection;
//   k_kacz_avg    one thread per displacement unknown: mean over its
//                 gather list (sub-region, LDS slot), fixed order;
//   k_kacz_spmv   one wavefront per row: y = S x or y = b - S x (pressure
//                 entries of y: b's, or zero);
//   k_kacz_elem   the element-wise steps of the elimination and the
//                 back-substitution of p.
#include "elh_internal.h"

namespace elh {

template <typename T> __device__ __forceinline__ T wave_sum(T v) {
  // xor butterfly: every lane ends with the same sum (each step adds a
  // pair in both orders, and IEEE addition commutes)
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

template <typename T>
__device__ __forceinline__ void kacz_cell(const KaczArgs<T>& K, int64_t cell, int* c) {
  c[0] = (int)(cell % K.n[0]);
  c[1] = (int)((cell / K.n[0]) % K.n[1]);
  c[2] = (int)(cell / ((int64_t)K.n[0] * K.n[1]));
}

template <typename T>
__global__ void __launch_bounds__(64) k_kacz_sweep(KaczArgs<T> K, const cx<T>* __restrict__ b,
                                                   const cx<T>* __restrict__ xin, cx<T>* __restrict__ scr) {
  extern __shared__ double kacz_lds[];
  cx<T>* X = (cx<T>*)kacz_lds;
  const int r = blockIdx.x, s = blockIdx.y, lane = threadIdx.x;
  const int br[3] = {r % K.nb[0], (r / K.nb[0]) % K.nb[1], r / (K.nb[0] * K.nb[1])};
  int lo[3], c0[3], c1[3];
  for (int a = 0; a < 3; ++a) {
    const bool ax = a < K.dim;
    lo[a] = ax ? br[a] * K.box - 2 : 0;
    c0[a] = ax ? br[a] * K.box : 0;
    c1[a] = ax ? min(c0[a] + K.box, K.n[a]) : 1;
  }
  const int e01 = K.E[0] * K.E[1], ee = e01 * K.E[2];
  const int64_t vb = (int64_t)s * K.vs;
  // private copy of the neighbourhood (zero outside the grid)
  for (int q = lane; q < K.ls; q += 64) {
    const int f = q / ee, e = q - f * ee;
    const int c[3] = {lo[0] + e % K.E[0], lo[1] + (e / K.E[0]) % K.E[1], lo[2] + e / e01};
    cx<T> v = czero<T>();
    if (xin && c[0] >= 0 && c[0] < K.n[0] && c[1] >= 0 && c[1] < K.n[1] && c[2] >= 0 && c[2] < K.n[2])
      v = xin[vb + f * K.fs + ((int64_t)c[2] * K.n[1] + c[1]) * K.n[0] + c[0]];
    X[q] = v;
  }
  __syncthreads();
  const cx<T>* bs = b + vb;
  const int q0 = lane, q1 = lane + 64;
  for (int k = 0; k < K.dim; ++k) {
    const int* dlk = K.dl + k * K.ns;
    const int d0 = q0 < K.ns ? dlk[q0] : 0, d1 = q1 < K.ns ? dlk[q1] : 0;
    for (int z = c0[2]; z < c1[2]; ++z)
      for (int y = c0[1]; y < c1[1]; ++y)
        for (int x = c0[0]; x < c1[0]; ++x) {
          const int c[3] = {x, y, z};
          if (c[k] == 0) continue;  // boundary face: not an unknown
          const int64_t row = k * K.fs + ((int64_t)z * K.n[1] + y) * K.n[0] + x;
          const T inv = K.inv[row];
          if (inv == T(0)) continue;
          const int lb = ((z - lo[2]) * K.E[1] + (y - lo[1])) * K.E[0] + (x - lo[0]);
          const cx<T>* vr = K.val + row * K.ns;
          const cx<T> a0 = q0 < K.ns ? vr[q0] : czero<T>();
          const cx<T> a1 = q1 < K.ns ? vr[q1] : czero<T>();
          const int l0 = lb + d0, l1 = lb + d1;
          cx<T> acc = a0 * X[l0];
          if (q1 < K.ns) acc += a1 * X[l1];
          const T dre = wave_sum(acc.re), dim_ = wave_sum(acc.im);
          const cx<T> res = bs[row] - mk(dre, dim_);
          const cx<T> coef = (K.omega * inv) * res;
          if (q0 < K.ns) X[l0] += coef * conj(a0);
          if (q1 < K.ns) X[l1] += coef * conj(a1);
        }
  }
  __syncthreads();
  cx<T>* out = scr + ((int64_t)s * K.nreg + r) * K.ls;
  for (int q = lane; q < K.ls; q += 64) out[q] = X[q];
}

template <typename T>
__global__ void k_kacz_avg(KaczArgs<T> K, const cx<T>* __restrict__ scr, cx<T>* __restrict__ x, int nrhs) {
  const int64_t nu = (int64_t)K.dim * K.fs;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nu * nrhs) return;
  const int s = (int)(i / nu);
  const int64_t j = i - (int64_t)s * nu;
  const int a = K.gptr[j], e = K.gptr[j + 1];
  if (a == e) return;  // reached by no row: keeps its value
  cx<T> sum = czero<T>();
  const cx<T>* sb = scr + (int64_t)s * K.nreg * K.ls;
  for (int q = a; q < e; ++q) sum += sb[(int64_t)K.gent[2 * q] * K.ls + K.gent[2 * q + 1]];
  const T cnt = T(e - a);
  x[(int64_t)s * K.vs + j] = mk(sum.re / cnt, sum.im / cnt);
}

template <typename T>
__global__ void __launch_bounds__(256) k_kacz_spmv(KaczArgs<T> K, const cx<T>* __restrict__ x,
                                                   const cx<T>* __restrict__ b, cx<T>* __restrict__ y, int nrhs) {
  const int lane = threadIdx.x & 63;
  const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (w >= K.vs * nrhs) return;  // whole wavefront
  const int s = (int)(w / K.vs);
  const int64_t row = w - (int64_t)s * K.vs;
  const int64_t vb = (int64_t)s * K.vs;
  const int64_t nu = (int64_t)K.dim * K.fs;
  if (row >= nu) {  // pressure entries
    if (lane == 0) y[vb + row] = b ? b[vb + row] : czero<T>();
    return;
  }
  const int k = (int)(row / K.fs);
  int c[3];
  kacz_cell(K, row - (int64_t)k * K.fs, c);
  cx<T> acc = czero<T>();
  if (c[k] > 0) {
    for (int q = lane; q < K.ns; q += 64) {
      const int* t = K.tab + (k * K.ns + q) * 4;
      const int l = t[0];
      const int cc[3] = {c[0] + t[1], c[1] + t[2], c[2] + t[3]};
      if (cc[0] < 0 || cc[0] >= K.n[0] || cc[1] < 0 || cc[1] >= K.n[1] || cc[2] < 0 || cc[2] >= K.n[2]) continue;
      if (cc[l] == 0) continue;
      acc += K.val[row * K.ns + q] * x[vb + l * K.fs + ((int64_t)cc[2] * K.n[1] + cc[1]) * K.n[0] + cc[0]];
    }
  }
  const T re = wave_sum(acc.re), im = wave_sum(acc.im);
  if (lane == 0) {
    const cx<T> v = mk(re, im);
    y[vb + row] = b ? b[vb + row] - v : v;
  }
}

// mode 0: out = [0; b_p / ap]            (input of A_up for the Schur rhs)
// mode 1: out = [b_u - y_u; 0]           (Schur right-hand side)
// mode 2: out_p = (b_p - y_p) / ap       (back-substitution, out_u untouched)
// ap = A_pp (forward) or conj(A_pp) (adjoint).
template <typename T>
__global__ void k_kacz_elem(int mode, int dim, int64_t fs, int64_t vs, int nrhs, const cx<T>* __restrict__ app,
                            int cj, const cx<T>* __restrict__ b, const cx<T>* __restrict__ y, cx<T>* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= vs * nrhs) return;
  const int64_t s = i / vs, e = i - s * vs;
  const int64_t nu = (int64_t)dim * fs;
  if (mode == 0) {
    if (e < nu) {
      out[i] = czero<T>();
    } else {
      cx<T> a = app[e - nu];
      if (cj) a = conj(a);
      out[i] = cdiv(b[i], a);
    }
  } else if (mode == 1) {
    out[i] = e < nu ? b[i] - y[i] : czero<T>();
  } else {
    if (e >= nu) {
      cx<T> a = app[e - nu];
      if (cj) a = conj(a);
      out[i] = cdiv(b[i] - y[i], a);
    }
  }
}

static inline int ngrid(int64_t n, int bs) { return (int)((n + bs - 1) / bs); }

template <typename T>
int launch_kacz_sweep(const KaczArgs<T>& K, const void* b, const void* xin, void* scr, int nrhs, hipStream_t st) {
  const size_t lds = (size_t)K.ls * sizeof(cx<T>);
  if (lds > KACZ_MAX_LDS || K.ns > 128 || nrhs > 65535) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(k_kacz_sweep<T>, dim3(K.nreg, nrhs), dim3(64), lds, st, K, (const cx<T>*)b,
                     (const cx<T>*)xin, (cx<T>*)scr);
  return (int)hipGetLastError();
}

template <typename T>
int launch_kacz_avg(const KaczArgs<T>& K, const void* scr, void* x, int nrhs, hipStream_t st) {
  const int64_t n = (int64_t)K.dim * K.fs * nrhs;
  hipLaunchKernelGGL(k_kacz_avg<T>, dim3(ngrid(n, 256)), dim3(256), 0, st, K, (const cx<T>*)scr, (cx<T>*)x, nrhs);
  return (int)hipGetLastError();
}

template <typename T>
int launch_kacz_spmv(const KaczArgs<T>& K, const void* x, const void* b, void* y, int nrhs, hipStream_t st) {
  const int64_t waves = K.vs * nrhs;
  hipLaunchKernelGGL(k_kacz_spmv<T>, dim3(ngrid(waves, 4)), dim3(256), 0, st, K, (const cx<T>*)x,
                     (const cx<T>*)b, (cx<T>*)y, nrhs);
  return (int)hipGetLastError();
}

template <typename T>
int launch_kacz_elem(int mode, int dim, int64_t fs, int64_t vs, int nrhs, const void* app, int cj, const void* b,
                     const void* y, void* out, hipStream_t st) {
  hipLaunchKernelGGL(k_kacz_elem<T>, dim3(ngrid(vs * nrhs, 256)), dim3(256), 0, st, mode, dim, fs, vs, nrhs,
                     (const cx<T>*)app, cj, (const cx<T>*)b, (const cx<T>*)y, (cx<T>*)out);
  return (int)hipGetLastError();
}

#define INST(T)                                                                                               \
  template int launch_kacz_sweep<T>(const KaczArgs<T>&, const void*, const void*, void*, int, hipStream_t); \
  template int launch_kacz_avg<T>(const KaczArgs<T>&, const void*, void*, int, hipStream_t);                \
  template int launch_kacz_spmv<T>(const KaczArgs<T>&, const void*, const void*, void*, int, hipStream_t);  \
  template int launch_kacz_elem<T>(int, int, int64_t, int64_t, int, const void*, int, const void*, const void*, \
                                   void*, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace elh
