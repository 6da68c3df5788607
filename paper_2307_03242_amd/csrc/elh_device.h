// Device-side building blocks of the elastic Helmholtz operator on the MAC
// grid: complex arithmetic, per-level arguments, bounds-aware loads and the
// point-wise evaluation of H^beta / H^beta_s / their adjoints.
//
// Operator (Section 3.1, eq. mixed-discretized; 3D form Section 5.3, eqs.
// dxSkew3D, massHO3D).  Row of u_k at a k-face P:
//   sum_l  D_l^T [ A_e(mu) * S^beta_l D_l u_k ]            (vector Laplacian)
//   - w2(P) * ( beta*rho_f(P) u_k(P)
//               + (1-beta)/(2d) * sum_{2d face nbrs Q} rho_f(Q) u_k(Q) )
//   + (p(right cell) - p(left cell)) / h                    (coupling)
// Row of p at cell c:  sum_k S^beta_k D_k u_k (c) + kappa(c) p(c).
// D_l: standard two-point difference (1/h)[-1 * 1]; S^beta_l: beta*I +
// (1-beta)*(1/4)[1 2 1] averaging over every axis other than l; A_e(mu):
// cell mu for the derivative of u_k along x_k, mean of the four cells
// around the edge otherwise (media clamped at the domain boundary);
// rho_f: mean of the two cells beside a face; w2 = omega^2 (1 - i gamma~),
// gamma~ = gamma (+ alpha when shifted) + absorbing-layer profile at P.
// Values outside the grid, and on boundary faces, are zero.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace elh {

template <typename T> struct cx { T re, im; };

template <typename T> __host__ __device__ inline cx<T> mk(T r, T i) { cx<T> z; z.re = r; z.im = i; return z; }
template <typename T> __host__ __device__ inline cx<T> czero() { return mk<T>(T(0), T(0)); }
template <typename T> __host__ __device__ inline cx<T> operator+(cx<T> a, cx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename T> __host__ __device__ inline cx<T> operator-(cx<T> a, cx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename T> __host__ __device__ inline cx<T> operator-(cx<T> a) { return mk(-a.re, -a.im); }
template <typename T> __host__ __device__ inline cx<T> operator*(cx<T> a, cx<T> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T> __host__ __device__ inline cx<T> operator*(T s, cx<T> a) { return mk(s * a.re, s * a.im); }
template <typename T> __host__ __device__ inline cx<T>& operator+=(cx<T>& a, cx<T> b) { a.re += b.re; a.im += b.im; return a; }
template <typename T> __host__ __device__ inline cx<T>& operator-=(cx<T>& a, cx<T> b) { a.re -= b.re; a.im -= b.im; return a; }
template <typename T> __host__ __device__ inline cx<T> conj(cx<T> a) { return mk(a.re, -a.im); }
template <typename T> __host__ __device__ inline T abs2(cx<T> a) { return a.re * a.re + a.im * a.im; }
template <typename T> __host__ __device__ inline cx<T> cdiv(cx<T> a, cx<T> b) {
  T d = b.re * b.re + b.im * b.im;
  return mk((a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d);
}

// Arguments describing one grid level in precision T.
template <typename T> struct LevelArgs {
  int n[3];          // cells along x_1, x_2, x_3 (n[2] = 1 in 2D)
  int64_t fs;        // cells per field = n[0]*n[1]*n[2]
  int64_t vs;        // complex entries per vector = (dim+1)*fs
  T h, ih;           // spacing and its inverse
  T beta;            // spread weight
  T omega2;          // omega^2
  T gam;             // gamma (+ alpha for the shifted operator)
  T abl_w, abl_amp;  // absorbing layer (physical width, amplitude)
  T abl_iw;          // 1 / abl_w (0 when there is no layer)
  const T* mu;       // cell media (fs each)
  const T* rho;
  const T* kap;      // 1/(lam+mu)
  const T* ablz;     // 3D: absorbing-layer term along x_3, amp*(delta/width)^2, at the
                     // cell centres (entries 0..n3-1) and at the lower faces (n3..2*n3-1)
};

template <int DIM> __device__ __forceinline__ bool in_grid(const int* n, const int* j) {
  bool ok = j[0] >= 0 && j[0] < n[0] && j[1] >= 0 && j[1] < n[1];
  if (DIM == 3) ok = ok && j[2] >= 0 && j[2] < n[2];
  return ok;
}

template <int DIM> __device__ __forceinline__ int64_t lin(const int* n, const int* j) {
  return DIM == 3 ? ((int64_t)j[2] * n[1] + j[1]) * n[0] + j[0] : (int64_t)j[1] * n[0] + j[0];
}

// Field f of x at storage index j (zero outside the grid or on a boundary
// face of a displacement field).
template <int DIM, typename T>
__device__ __forceinline__ cx<T> ldf(const cx<T>* __restrict__ x, const LevelArgs<T>& L, int f, const int* j) {
  if (!in_grid<DIM>(L.n, j)) return czero<T>();
  if (f < DIM && j[f] == 0) return czero<T>();
  return x[f * L.fs + lin<DIM>(L.n, j)];
}

template <int DIM, typename T>
__device__ __forceinline__ T ldm(const T* __restrict__ m, const int* n, const int* j) {
  int c[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) c[a] = j[a] < 0 ? 0 : (j[a] >= n[a] ? n[a] - 1 : j[a]);
  return m[lin<DIM>(n, c)];
}

// Absorbing-layer attenuation at physical position xp[] (reading of the
// layer of Section 5: quadratic ramp over the layer width).
template <int DIM, typename T>
__device__ __forceinline__ T abl_gamma(const LevelArgs<T>& L, const T* xp) {
  if (L.abl_w <= T(0) || L.abl_amp == T(0)) return T(0);
  T s = T(0);
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    T len = L.n[a] * L.h;
    T d = (L.abl_w - xp[a] > T(0) ? L.abl_w - xp[a] : T(0)) +
          (xp[a] - (len - L.abl_w) > T(0) ? xp[a] - (len - L.abl_w) : T(0));
    T r = d * L.abl_iw;
    s += r * r;
  }
  return L.abl_amp * s;
}

// omega^2 (1 - i gamma~) at the u_k face with storage index j.
template <int DIM, typename T>
__device__ __forceinline__ cx<T> mass_factor(const LevelArgs<T>& L, int k, const int* j) {
  T xp[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) xp[a] = (a == k ? T(j[a]) : T(j[a]) + T(0.5)) * L.h;
  T g = L.gam + abl_gamma<DIM, T>(L, xp);
  return mk(L.omega2, -L.omega2 * g);
}

// rho averaged onto the u_k face j (j[k] in 1..n_k-1).
template <int DIM, typename T>
__device__ __forceinline__ T rho_face(const LevelArgs<T>& L, int k, const int* j) {
  int c[3] = {j[0], j[1], j[2]};
  T a = L.rho[lin<DIM>(L.n, c)];
  c[k] -= 1;
  return T(0.5) * (a + L.rho[lin<DIM>(L.n, c)]);
}

// mu averaged onto the edge of u_k's derivative along x_l (l != k): k-face
// index e[k], l-face index e[l] (0..n_l), cell index along the third axis.
template <int DIM, typename T>
__device__ __forceinline__ T mu_edge(const LevelArgs<T>& L, int k, int l, const int* e) {
  int c[3] = {e[0], e[1], e[2]};
  T s = T(0);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      c[k] = e[k] - 1 + a;
      c[l] = e[l] - 1 + b;
      s += ldm<DIM>(L.mu, L.n, c);
    }
  return T(0.25) * s;
}

__device__ __forceinline__ double w121(int o) { return o == 0 ? 0.5 : 0.25; }

// Forward beta-spread flux of u_k along x_l at flux index q along l:
//   l == k: cell q,   difference u_k(face q+1) - u_k(face q);
//   l != k: l-face q, difference u_k(cell q) - u_k(cell q-1);
// transverse coordinates t[] (u_k's own grid), spread over axes != l.
template <int DIM, typename T>
__device__ __forceinline__ cx<T> spread_flux(const cx<T>* __restrict__ x, const LevelArgs<T>& L, int k, int l,
                                             int q, const int* t) {
  const int hi = (l == k) ? q + 1 : q;
  const int lo = hi - 1;
  cx<T> centre, spread = czero<T>();
  int j[3] = {t[0], t[1], t[2]};
  int ax[2] = {0, 0};
  int na = 0;
#pragma unroll
  for (int a = 0; a < DIM; ++a)
    if (a != l) ax[na++] = a;
  {
    j[l] = hi;
    cx<T> vh = ldf<DIM>(x, L, k, j);
    j[l] = lo;
    centre = vh - ldf<DIM>(x, L, k, j);
  }
  if (DIM == 2) {
#pragma unroll
    for (int o = -1; o <= 1; ++o) {
      j[ax[0]] = t[ax[0]] + o;
      j[l] = hi;
      cx<T> vh = ldf<DIM>(x, L, k, j);
      j[l] = lo;
      spread += T(w121(o)) * (vh - ldf<DIM>(x, L, k, j));
    }
  } else {
#pragma unroll
    for (int o0 = -1; o0 <= 1; ++o0)
#pragma unroll
      for (int o1 = -1; o1 <= 1; ++o1) {
        j[ax[0]] = t[ax[0]] + o0;
        j[ax[1]] = t[ax[1]] + o1;
        j[l] = hi;
        cx<T> vh = ldf<DIM>(x, L, k, j);
        j[l] = lo;
        spread += T(w121(o0) * w121(o1)) * (vh - ldf<DIM>(x, L, k, j));
      }
  }
  return L.ih * (L.beta * centre + (T(1) - L.beta) * spread);
}

// Adjoint helper: g(q, t) = A_e(mu) * (standard difference of u_k along l)
// at flux index q along l and flux-grid transverse index t (zero outside).
template <int DIM, typename T>
__device__ __forceinline__ cx<T> mu_flux(const cx<T>* __restrict__ x, const LevelArgs<T>& L, int k, int l, int q,
                                         const int* t) {
  int j[3] = {t[0], t[1], t[2]};
  // flux grid along l: cells 0..n_l-1 (l == k) or faces 0..n_l (l != k);
  // transverse: u_k's grid (interior faces along k, cells otherwise).
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    if (a == l) continue;
    if (t[a] < 0 || t[a] >= L.n[a]) return czero<T>();
    if (a == k && t[a] == 0) return czero<T>();
  }
  if (l == k) {
    if (q < 0 || q >= L.n[l]) return czero<T>();
  } else {
    if (q < 0 || q > L.n[l]) return czero<T>();
  }
  const int hi = (l == k) ? q + 1 : q;
  j[l] = hi;
  cx<T> d = ldf<DIM>(x, L, k, j);
  j[l] = hi - 1;
  d = d - ldf<DIM>(x, L, k, j);
  T m;
  if (l == k) {
    j[l] = q;
    m = L.mu[lin<DIM>(L.n, j)];
  } else {
    j[l] = q;
    m = mu_edge<DIM>(L, k, l, j);
  }
  return (m * L.ih) * d;
}

// Adjoint spread of a flux-grid quantity: beta*g + (1-beta)*A A g over the
// axes other than l.
template <int DIM, typename T>
__device__ __forceinline__ cx<T> spread_mu_flux(const cx<T>* __restrict__ x, const LevelArgs<T>& L, int k, int l,
                                                int q, const int* t) {
  cx<T> centre = mu_flux<DIM>(x, L, k, l, q, t);
  cx<T> spread = czero<T>();
  int ax[2] = {0, 0};
  int na = 0;
#pragma unroll
  for (int a = 0; a < DIM; ++a)
    if (a != l) ax[na++] = a;
  int tt[3] = {t[0], t[1], t[2]};
  if (DIM == 2) {
#pragma unroll
    for (int o = -1; o <= 1; ++o) {
      tt[ax[0]] = t[ax[0]] + o;
      spread += T(w121(o)) * mu_flux<DIM>(x, L, k, l, q, tt);
    }
  } else {
#pragma unroll
    for (int o0 = -1; o0 <= 1; ++o0)
#pragma unroll
      for (int o1 = -1; o1 <= 1; ++o1) {
        tt[ax[0]] = t[ax[0]] + o0;
        tt[ax[1]] = t[ax[1]] + o1;
        spread += T(w121(o0) * w121(o1)) * mu_flux<DIM>(x, L, k, l, q, tt);
      }
  }
  return L.beta * centre + (T(1) - L.beta) * spread;
}

// Spread (beta*I + (1-beta) A A over the axes != k) of the pressure at
// cell c (zero outside).
template <int DIM, typename T>
__device__ __forceinline__ cx<T> spread_p(const cx<T>* __restrict__ x, const LevelArgs<T>& L, int k, const int* c) {
  cx<T> centre = ldf<DIM>(x, L, DIM, c);
  cx<T> spread = czero<T>();
  int ax[2] = {0, 0};
  int na = 0;
#pragma unroll
  for (int a = 0; a < DIM; ++a)
    if (a != k) ax[na++] = a;
  int j[3] = {c[0], c[1], c[2]};
  if (DIM == 2) {
#pragma unroll
    for (int o = -1; o <= 1; ++o) {
      j[ax[0]] = c[ax[0]] + o;
      spread += T(w121(o)) * ldf<DIM>(x, L, DIM, j);
    }
  } else {
#pragma unroll
    for (int o0 = -1; o0 <= 1; ++o0)
#pragma unroll
      for (int o1 = -1; o1 <= 1; ++o1) {
        j[ax[0]] = c[ax[0]] + o0;
        j[ax[1]] = c[ax[1]] + o1;
        spread += T(w121(o0) * w121(o1)) * ldf<DIM>(x, L, DIM, j);
      }
  }
  return L.beta * centre + (T(1) - L.beta) * spread;
}

// Row of u_k at face P (P[k] in 1..n_k-1) of H (ADJ = false) or H^H.
template <int DIM, bool ADJ, typename T>
__device__ cx<T> eval_u(const cx<T>* __restrict__ x, const LevelArgs<T>& L, int k, const int* P) {
  cx<T> acc = czero<T>();
  // vector Laplacian
#pragma unroll
  for (int l = 0; l < DIM; ++l) {
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const T sg = side == 0 ? T(1) : T(-1);
      int q = (l == k) ? P[k] - 1 + side : P[l] + side;
      cx<T> term;
      if (!ADJ) {
        T m;
        if (l == k) {
          int c[3] = {P[0], P[1], P[2]};
          c[k] = q;
          m = L.mu[lin<DIM>(L.n, c)];
        } else {
          int e[3] = {P[0], P[1], P[2]};
          e[l] = q;
          m = mu_edge<DIM>(L, k, l, e);
        }
        term = m * spread_flux<DIM>(x, L, k, l, q, P);
      } else {
        term = spread_mu_flux<DIM>(x, L, k, l, q, P);
      }
      acc += (sg * L.ih) * term;
    }
  }
  // mass
  {
    const T cn = (T(1) - L.beta) / T(2 * DIM);
    cx<T> mfP = mass_factor<DIM>(L, k, P);
    T rP = rho_face<DIM>(L, k, P);
    cx<T> uP = ldf<DIM>(x, L, k, P);
    cx<T> m = ADJ ? (L.beta * (conj(mfP) * uP)) : ((L.beta * rP) * uP);
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
      for (int s = -1; s <= 1; s += 2) {
        int Q[3] = {P[0], P[1], P[2]};
        Q[a] += s;
        if (!in_grid<DIM>(L.n, Q)) continue;
        if (Q[k] == 0) continue;
        cx<T> uQ = x[k * L.fs + lin<DIM>(L.n, Q)];
        if (ADJ)
          m += cn * (conj(mass_factor<DIM>(L, k, Q)) * uQ);
        else
          m += (cn * rho_face<DIM>(L, k, Q)) * uQ;
      }
    acc -= ADJ ? (rP * m) : (mfP * m);
  }
  // coupling with p
  {
    int c[3] = {P[0], P[1], P[2]};
    if (!ADJ) {
      cx<T> pr = ldf<DIM>(x, L, DIM, c);
      c[k] -= 1;
      acc += L.ih * (pr - ldf<DIM>(x, L, DIM, c));
    } else {
      c[k] -= 1;
      cx<T> pl = spread_p<DIM>(x, L, k, c);
      c[k] += 1;
      acc += L.ih * (pl - spread_p<DIM>(x, L, k, c));
    }
  }
  return acc;
}

// Row of p at cell c.
template <int DIM, bool ADJ, typename T>
__device__ cx<T> eval_p(const cx<T>* __restrict__ x, const LevelArgs<T>& L, const int* c) {
  cx<T> acc = L.kap[lin<DIM>(L.n, c)] * ldf<DIM>(x, L, DIM, c);
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    if (!ADJ) {
      acc += spread_flux<DIM>(x, L, k, k, c[k], c);
    } else {
      int j[3] = {c[0], c[1], c[2]};
      cx<T> a = ldf<DIM>(x, L, k, j);
      j[k] += 1;
      acc += L.ih * (a - ldf<DIM>(x, L, k, j));
    }
  }
  return acc;
}

}  // namespace elh
