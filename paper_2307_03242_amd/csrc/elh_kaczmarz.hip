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
//                 DPP sum gives a_i . x (wave-uniform) and every lane applies
//                 its slots' share of the projection; the next row's entries
//                 are loaded during the current projection;
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

// DPP move with row mask RM; lanes of disabled rows read zero.
template <int CTRL, int RM> __device__ __forceinline__ float dpp0(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, RM, 0xf, false));
}
template <int CTRL, int RM> __device__ __forceinline__ double dpp0(double v) {
  const long long u = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xffffffffll), CTRL, RM, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, RM, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float lane63(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}
__device__ __forceinline__ double lane63(double v) {
  const long long u = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffll), 63);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), 63);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
// Sum over the 64 lanes, wave-uniform result: pairs and quads (quad
// permutes), rows of 16 (row rotates by 4 and 8), then the row broadcasts
// carry rows 0+1 and 2+3 and finally all four rows into lane 63.
template <typename T> __device__ __forceinline__ T wave_total(T v) {
  v += dpp0<0xb1, 0xf>(v);   // quad_perm [1,0,3,2]
  v += dpp0<0x4e, 0xf>(v);   // quad_perm [2,3,0,1]
  v += dpp0<0x124, 0xf>(v);  // row_ror:4
  v += dpp0<0x128, 0xf>(v);  // row_ror:8
  v += dpp0<0x142, 0xa>(v);  // row_bcast:15 into rows 1, 3
  v += dpp0<0x143, 0xc>(v);  // row_bcast:31 into rows 2, 3
  return lane63(v);
}

// Raw buffer resource and vector loads through it (wave-uniform addresses
// stay in the vector memory pipeline, counted with the other loads).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t kacz_rsrc(const void* p, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0,
                                           (int)(bytes > 0x7fffffffll ? 0x7fffffffll : bytes), 0x00020000);
}
template <typename V> __device__ __forceinline__ V kacz_load(__amdgpu_buffer_rsrc_t r, int off);
template <> __device__ __forceinline__ float kacz_load<float>(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <> __device__ __forceinline__ double kacz_load<double>(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <> __device__ __forceinline__ cx<float> kacz_load<cx<float>>(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(cx<float>, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <> __device__ __forceinline__ cx<double> kacz_load<cx<double>>(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(cx<double>, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
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
  const int q0 = lane, q1 = lane + 64;
  const bool has1 = q1 < K.ns;
  // rows of the sub-region in ascending global order: an odometer over
  // (field, x_3, x_2, x_1) of the box.  Boundary faces (not unknowns) hold
  // zero entries and 1/||a||^2 = 0, so their projection changes nothing and
  // every box position is taken in turn.  Four register sets form a ring:
  // the entries, 1/||a||^2 and b_i of the rows three ahead are in flight
  // while a row is projected.  Every lane loads unconditionally (the row
  // table carries 128 zero slots of padding at its end) and surplus slots
  // are multiplied by zero, so the loop is straight-line.
  const T m0 = q0 < K.ns ? T(1) : T(0), m1 = has1 ? T(1) : T(0);
  int dls[3][2];
  for (int k = 0; k < 3; ++k) {
    dls[k][0] = k < K.dim && q0 < K.ns ? K.dl[k * K.ns + q0] : 0;
    dls[k][1] = k < K.dim && has1 ? K.dl[k * K.ns + q1] : 0;
  }
  const int w0 = c1[0] - c0[0], w1 = c1[1] - c0[1], w2 = c1[2] - c0[2];
  const int nt = K.dim * w0 * w1 * w2;
  const __amdgpu_buffer_rsrc_t rb = kacz_rsrc(b + vb, K.vs * (int64_t)sizeof(cx<T>));
  const __amdgpu_buffer_rsrc_t ri = kacz_rsrc(K.inv, (int64_t)K.dim * K.fs * (int64_t)sizeof(T));
  struct Row {
    int c[3], k;
    cx<T> a0, a1, bi;
    T inv;
  };
  auto step = [&](Row& r) {
    if (++r.c[0] < c1[0]) return;
    r.c[0] = c0[0];
    if (++r.c[1] < c1[1]) return;
    r.c[1] = c0[1];
    if (++r.c[2] < c1[2]) return;
    r.c[2] = c0[2];
    ++r.k;
  };
  // past the last row the odometer's field index runs to dim: fetch() clamps
  // it, and those rows are never projected
  auto fetch = [&](Row& r) {
    const int row = min(r.k, K.dim - 1) * (int)K.fs + (r.c[2] * K.n[1] + r.c[1]) * K.n[0] + r.c[0];
    const cx<T>* vr = K.val + (int64_t)row * K.ns;
    const cx<T> v0 = vr[q0], v1 = vr[q1];
    r.a0 = mk(v0.re * m0, v0.im * m0);
    r.a1 = mk(v1.re * m1, v1.im * m1);
    r.bi = kacz_load<cx<T>>(rb, row * (int)sizeof(cx<T>));
    r.inv = kacz_load<T>(ri, row * (int)sizeof(T));
  };
  auto project = [&](const Row& r) {
    const int lb = ((r.c[2] - lo[2]) * K.E[1] + (r.c[1] - lo[1])) * K.E[0] + (r.c[0] - lo[0]);
    const int l0 = lb + dls[r.k][0], l1 = lb + dls[r.k][1];
    const cx<T> acc = r.a0 * X[l0] + r.a1 * X[l1];
    const T dre = wave_total(acc.re), dim_ = wave_total(acc.im);
    const cx<T> coef = (K.omega * r.inv) * (r.bi - mk(dre, dim_));
    // surplus lanes point at the row's own slot: they must not store
    if (q0 < K.ns) X[l0] += coef * conj(r.a0);
    if (has1) X[l1] += coef * conj(r.a1);
  };
  Row R[4];
  R[0].c[0] = c0[0]; R[0].c[1] = c0[1]; R[0].c[2] = c0[2]; R[0].k = 0;
#pragma unroll
  for (int j = 1; j < 4; ++j) {
    R[j].c[0] = R[j - 1].c[0]; R[j].c[1] = R[j - 1].c[1]; R[j].c[2] = R[j - 1].c[2]; R[j].k = R[j - 1].k;
    step(R[j]);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) fetch(R[j]);
  for (int i = 0; i < nt; i += 4) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (i + j < nt) project(R[j]);
      step(R[j]); step(R[j]); step(R[j]); step(R[j]);
      fetch(R[j]);
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
  ELH_LAUNCH(k_kacz_sweep<T>, dim3(K.nreg, nrhs), dim3(64), lds, st, K, (const cx<T>*)b,
                     (const cx<T>*)xin, (cx<T>*)scr);
  return (int)hipGetLastError();
}

template <typename T>
int launch_kacz_avg(const KaczArgs<T>& K, const void* scr, void* x, int nrhs, hipStream_t st) {
  const int64_t n = (int64_t)K.dim * K.fs * nrhs;
  ELH_LAUNCH(k_kacz_avg<T>, dim3(ngrid(n, 256)), dim3(256), 0, st, K, (const cx<T>*)scr, (cx<T>*)x, nrhs);
  return (int)hipGetLastError();
}

template <typename T>
int launch_kacz_spmv(const KaczArgs<T>& K, const void* x, const void* b, void* y, int nrhs, hipStream_t st) {
  const int64_t waves = K.vs * nrhs;
  ELH_LAUNCH(k_kacz_spmv<T>, dim3(ngrid(waves, 4)), dim3(256), 0, st, K, (const cx<T>*)x,
                     (const cx<T>*)b, (cx<T>*)y, nrhs);
  return (int)hipGetLastError();
}

template <typename T>
int launch_kacz_elem(int mode, int dim, int64_t fs, int64_t vs, int nrhs, const void* app, int cj, const void* b,
                     const void* y, void* out, hipStream_t st) {
  ELH_LAUNCH(k_kacz_elem<T>, dim3(ngrid(vs * nrhs, 256)), dim3(256), 0, st, mode, dim, fs, vs, nrhs,
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
