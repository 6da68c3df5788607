// Reference-structured gfx950 kernels: operator apply / residual (all
// levels, 2D and 3D, forward and adjoint), red-black full Vanka, MAC
// restriction and prolongation, media setup and Krylov vector operations.
// The 3D wavefront-march stencil kernels (levels from 16^3) live in
// elh_stencil3d_wave.hip.
#include "elh_device.h"
#include "elh_internal.h"

namespace elh {

// ---------------------------------------------------------------------------
// apply / residual: one thread per cell, the cell's left faces and pressure
// ---------------------------------------------------------------------------
template <int DIM, bool ADJ, typename T>
__global__ void __launch_bounds__(256) k_apply(LevelArgs<T> L, const cx<T>* __restrict__ x,
                                                const cx<T>* __restrict__ b, cx<T>* __restrict__ y,
                                                int nrhs) {
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (cell >= L.fs || s >= nrhs) return;
  int c[3];
  c[0] = (int)(cell % L.n[0]);
  c[1] = (int)((cell / L.n[0]) % L.n[1]);
  c[2] = (int)(cell / ((int64_t)L.n[0] * L.n[1]));
  const cx<T>* xs = x + s * L.vs;
  cx<T>* ys = y + s * L.vs;
  const cx<T>* bs = b ? b + s * L.vs : nullptr;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    cx<T> v = czero<T>();
    if (c[k] > 0) {
      v = eval_u<DIM, ADJ>(xs, L, k, c);
      if (bs) v = bs[k * L.fs + cell] - v;
    }
    ys[k * L.fs + cell] = v;
  }
  cx<T> v = eval_p<DIM, ADJ>(xs, L, c);
  if (bs) v = bs[DIM * L.fs + cell] - v;
  ys[DIM * L.fs + cell] = v;
}

template <typename T>
int launch_apply(const LevelArgs<T>& L, int dim, bool adj, const void* x, const void* b, void* y, int nrhs,
                 hipStream_t st) {
  dim3 blk(256), grd((unsigned)((L.fs + 255) / 256), nrhs);
  const cx<T>* xp = (const cx<T>*)x;
  const cx<T>* bp = (const cx<T>*)b;
  cx<T>* yp = (cx<T>*)y;
  if (dim == 3) {
    if (adj) ELH_LAUNCH((k_apply<3, true, T>), grd, blk, 0, st, L, xp, bp, yp, nrhs);
    else ELH_LAUNCH((k_apply<3, false, T>), grd, blk, 0, st, L, xp, bp, yp, nrhs);
  } else {
    if (adj) ELH_LAUNCH((k_apply<2, true, T>), grd, blk, 0, st, L, xp, bp, yp, nrhs);
    else ELH_LAUNCH((k_apply<2, false, T>), grd, blk, 0, st, L, xp, bp, yp, nrhs);
  }
  return (int)hipGetLastError();
}
template int launch_apply<double>(const LevelArgs<double>&, int, bool, const void*, const void*, void*, int,
                                  hipStream_t);
template int launch_apply<float>(const LevelArgs<float>&, int, bool, const void*, const void*, void*, int,
                                 hipStream_t);

// ---------------------------------------------------------------------------
// red-black full Vanka: cell block of H_s (Section 2.3, Section 3.2 remark)
// ---------------------------------------------------------------------------
// Entries of the forward shifted operator on the DOFs of cell c: for each
// component k the 2x2 block B_k over its left (face c_k) and right (face
// c_k+1) faces, the coupling column g_k = (+1/h, -1/h) (u rows, p column),
// the divergence row d_k = (-s0/h, +s0/h) and kappa.  s0 = beta +
// (1-beta)/2^(d-1) is the centre weight of the spread difference and
// s1 = (1-beta)/4 * (1/2)^(d-2) the weight of a neighbouring face of the
// same component in the spread along x_k of a transverse difference.
template <int DIM, typename T>
__device__ void vanka_block(const LevelArgs<T>& L, int k, const int* c, cx<T>* B /*LL,LR,RL,RR*/) {
  const T s0 = L.beta + (T(1) - L.beta) / T(DIM == 3 ? 4 : 2);
  const T s1 = (T(1) - L.beta) * T(0.25) * T(DIM == 3 ? 0.5 : 1.0);
  const T ih2 = L.ih * L.ih;
  const T cn = (T(1) - L.beta) / T(2 * DIM);
  int F[2][3];
#pragma unroll
  for (int sd = 0; sd < 2; ++sd) {
    F[sd][0] = c[0]; F[sd][1] = c[1]; F[sd][2] = c[2];
    F[sd][k] = c[k] + sd;
  }
  const bool okL = c[k] >= 1, okR = c[k] + 1 <= L.n[k] - 1;
  const T muc = L.mu[lin<DIM>(L.n, c)];
  T sum_e[2] = {T(0), T(0)};
  T rf[2] = {T(0), T(0)};
  cx<T> mf[2];
#pragma unroll
  for (int sd = 0; sd < 2; ++sd) {
    const bool ok = sd == 0 ? okL : okR;
    if (!ok) { mf[sd] = czero<T>(); continue; }
#pragma unroll
    for (int l = 0; l < DIM; ++l) {
      if (l == k) continue;
      int e[3] = {F[sd][0], F[sd][1], F[sd][2]};
      e[l] = c[l];
      sum_e[sd] += mu_edge<DIM>(L, k, l, e);
      e[l] = c[l] + 1;
      sum_e[sd] += mu_edge<DIM>(L, k, l, e);
    }
    rf[sd] = rho_face<DIM>(L, k, F[sd]);
    mf[sd] = mass_factor<DIM>(L, k, F[sd]);
  }
  // diagonal entries: cells on both sides of the face along k
  {
    int cl[3] = {c[0], c[1], c[2]};
    cl[k] = c[k] - 1;
    T muL = okL ? L.mu[lin<DIM>(L.n, cl)] : T(0);
    int cr[3] = {c[0], c[1], c[2]};
    cr[k] = c[k] + 1;
    T muR = okR ? L.mu[lin<DIM>(L.n, cr)] : T(0);
    B[0] = okL ? mk(s0 * ih2 * (muL + muc + sum_e[0]), T(0)) - (L.beta * rf[0]) * mf[0] : mk(T(1), T(0));
    B[3] = okR ? mk(s0 * ih2 * (muc + muR + sum_e[1]), T(0)) - (L.beta * rf[1]) * mf[1] : mk(T(1), T(0));
  }
  if (okL && okR) {
    B[1] = mk(-muc * s0 * ih2 + s1 * ih2 * sum_e[0], T(0)) - (cn * rf[1]) * mf[0];
    B[2] = mk(-muc * s0 * ih2 + s1 * ih2 * sum_e[1], T(0)) - (cn * rf[0]) * mf[1];
  } else {
    B[1] = czero<T>();
    B[2] = czero<T>();
  }
}

template <int DIM, bool ADJ, typename T>
__global__ void __launch_bounds__(256) k_vanka(LevelArgs<T> L, const cx<T>* __restrict__ r, cx<T>* __restrict__ x,
                                                int colour, T w, int nrhs) {
  // one thread per cell of the active colour: thread i takes the i-th
  // such cell of its x_1 line (lines hold ceil/floor(n_1/2) of them)
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  const int half = (L.n[0] + 1) / 2;
  const int64_t lines = L.fs / L.n[0];
  if (id >= lines * half || s >= nrhs) return;
  const int64_t line = id / half;
  int c[3];
  c[1] = (int)(line % L.n[1]);
  c[2] = (int)(line / L.n[1]);
  const int par = (colour + c[1] + c[2]) & 1;  // parity of c_1 on this line
  c[0] = 2 * (int)(id % half) + par;
  if (c[0] >= L.n[0]) return;
  const int64_t cell = line * L.n[0] + c[0];
  const cx<T>* rs = r + s * L.vs;
  cx<T>* xs = x + s * L.vs;
  const T s0 = L.beta + (T(1) - L.beta) / T(DIM == 3 ? 4 : 2);
  // per component: Binv r and Binv g
  cx<T> yr[DIM][2], yg[DIM][2];
  cx<T> schur = mk(L.kap[cell], T(0));
  cx<T> rp = rs[DIM * L.fs + cell];
  int64_t idx[DIM][2];
  bool ok[DIM][2];
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    cx<T> B[4];
    vanka_block<DIM, T>(L, k, c, B);
    ok[k][0] = c[k] >= 1;
    ok[k][1] = c[k] + 1 <= L.n[k] - 1;
    int j[3] = {c[0], c[1], c[2]};
    idx[k][0] = k * L.fs + cell;
    j[k] = c[k] + 1;
    idx[k][1] = ok[k][1] ? k * L.fs + lin<DIM>(L.n, j) : 0;
    cx<T> g[2], d[2];
    g[0] = mk(ok[k][0] ? L.ih : T(0), T(0));
    g[1] = mk(ok[k][1] ? -L.ih : T(0), T(0));
    d[0] = mk(ok[k][0] ? -s0 * L.ih : T(0), T(0));
    d[1] = mk(ok[k][1] ? s0 * L.ih : T(0), T(0));
    if (ADJ) {  // block of H^H = conjugate transpose
      cx<T> t = B[1];
      B[0] = conj(B[0]); B[3] = conj(B[3]);
      B[1] = conj(B[2]); B[2] = conj(t);
      cx<T> g0 = g[0], g1 = g[1];
      g[0] = conj(d[0]); g[1] = conj(d[1]);
      d[0] = conj(g0); d[1] = conj(g1);
    }
    cx<T> rk[2];
    rk[0] = ok[k][0] ? rs[idx[k][0]] : czero<T>();
    rk[1] = ok[k][1] ? rs[idx[k][1]] : czero<T>();
    const cx<T> det = B[0] * B[3] - B[1] * B[2];
    const T id2 = T(1) / abs2(det);
    const cx<T> rdet = mk(det.re * id2, -det.im * id2);  // 1/det
    const cx<T> inv00 = B[3] * rdet, inv01 = -(B[1] * rdet), inv10 = -(B[2] * rdet), inv11 = B[0] * rdet;
    yr[k][0] = inv00 * rk[0] + inv01 * rk[1];
    yr[k][1] = inv10 * rk[0] + inv11 * rk[1];
    yg[k][0] = inv00 * g[0] + inv01 * g[1];
    yg[k][1] = inv10 * g[0] + inv11 * g[1];
    rp -= d[0] * yr[k][0] + d[1] * yr[k][1];
    schur -= d[0] * yg[k][0] + d[1] * yg[k][1];
  }
  const T is2 = T(1) / abs2(schur);
  cx<T> dp = rp * mk(schur.re * is2, -schur.im * is2);
  xs[DIM * L.fs + cell] += w * dp;
#pragma unroll
  for (int k = 0; k < DIM; ++k)
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
      if (ok[k][sd]) xs[idx[k][sd]] += w * (yr[k][sd] - yg[k][sd] * dp);
}

// 3D Vanka half-sweep with the block media formed from the 19 cells of the
// 3x3x3 box around the cell that the blocks touch (corners excluded).  The
// four edge means around a k-face between cells L and C sum to
//   mu_L + mu_C + (1/4) (N4(L) + N4(C)),
// N4(X) the sum of mu over the four neighbours of X across the axes other
// than k (indices clamped to the grid, like the edge means of the
// operator).  The absorbing-layer profile is summed per axis: centre and
// both face positions once per cell.  Same blocks, Schur complement and
// update as k_vanka.
template <bool ADJ, bool WR, typename T>
__global__ void __launch_bounds__(256) k_vanka3(LevelArgs<T> L, const cx<T>* __restrict__ r, cx<T>* __restrict__ x,
                                                 int colour, T w, int nrhs) {
  // WR (first half-sweep from a zero iterate): x holds no values yet; the
  // corrections are written, not added, and every entry that no block of
  // this colour writes is set to zero here: the cell's own boundary faces,
  // and the pressure and boundary faces of its two x_1 neighbours (the other
  // colour; each of those has at least one neighbour of this colour).
  // 32-bit index arithmetic (the launcher checks the cell count fits)
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  const int n0 = L.n[0], n1 = L.n[1];
  const int half = (n0 + 1) / 2;
  const int lines = n1 * L.n[2];
  if (id >= lines * half || s >= nrhs) return;
  const int line = id / half;
  int c[3];
  c[1] = line % n1;
  c[2] = line / n1;
  const int par = (colour + c[1] + c[2]) & 1;
  c[0] = 2 * (id - line * half) + par;
  if (c[0] >= n0) return;
  const int64_t cell = (int64_t)line * n0 + c[0];
  const int64_t st[3] = {1, n0, (int64_t)n0 * n1};
  // clamped neighbour coordinates and their offsets from the cell
  int64_t om[3], op[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    om[a] = c[a] > 0 ? -st[a] : 0;
    op[a] = c[a] < L.n[a] - 1 ? st[a] : 0;
  }
  const T* __restrict__ M = L.mu + cell;
  const T mc = M[0];
  const T mx0 = M[om[0]], mx1 = M[op[0]], my0 = M[om[1]], my1 = M[op[1]], mz0 = M[om[2]], mz1 = M[op[2]];
  const T mxy00 = M[om[0] + om[1]], mxy01 = M[om[0] + op[1]], mxy10 = M[op[0] + om[1]], mxy11 = M[op[0] + op[1]];
  const T mxz00 = M[om[0] + om[2]], mxz01 = M[om[0] + op[2]], mxz10 = M[op[0] + om[2]], mxz11 = M[op[0] + op[2]];
  const T myz00 = M[om[1] + om[2]], myz01 = M[om[1] + op[2]], myz10 = M[op[1] + om[2]], myz11 = M[op[1] + op[2]];
  // N4 over the axes other than k at L = c - e_k, C = c, R = c + e_k
  T n4[3][3];
  n4[0][0] = mxy00 + mxy01 + mxz00 + mxz01;
  n4[0][1] = my0 + my1 + mz0 + mz1;
  n4[0][2] = mxy10 + mxy11 + mxz10 + mxz11;
  n4[1][0] = mxy00 + mxy10 + myz00 + myz01;
  n4[1][1] = mx0 + mx1 + mz0 + mz1;
  n4[1][2] = mxy01 + mxy11 + myz10 + myz11;
  n4[2][0] = mxz00 + mxz10 + myz00 + myz10;
  n4[2][1] = mx0 + mx1 + my0 + my1;
  n4[2][2] = mxz01 + mxz11 + myz01 + myz11;
  const T mL[3] = {mx0, my0, mz0}, mR[3] = {mx1, my1, mz1};
  const T* __restrict__ RH = L.rho + cell;
  const T rc = RH[0];
  const T rL[3] = {RH[om[0]], RH[om[1]], RH[om[2]]}, rR[3] = {RH[op[0]], RH[op[1]], RH[op[2]]};
  // absorbing layer per axis: at the cell centre and at both faces
  T acen[3] = {T(0), T(0), T(0)}, alo[3] = {T(0), T(0), T(0)}, ahi[3] = {T(0), T(0), T(0)};
  if (L.abl_w > T(0) && L.abl_amp != T(0)) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const T len = L.n[a] * L.h;
      auto prof = [&](T xp) {
        T d = (L.abl_w - xp > T(0) ? L.abl_w - xp : T(0)) + (xp - (len - L.abl_w) > T(0) ? xp - (len - L.abl_w) : T(0));
        T q = d * L.abl_iw;
        return L.abl_amp * (q * q);
      };
      acen[a] = prof((T(c[a]) + T(0.5)) * L.h);
      alo[a] = prof(T(c[a]) * L.h);
      ahi[a] = prof(T(c[a] + 1) * L.h);
    }
  }
  const T asum = acen[0] + acen[1] + acen[2];
  const cx<T>* rs = r + s * L.vs;
  cx<T>* xs = x + s * L.vs;
  const T s0 = L.beta + (T(1) - L.beta) / T(4);
  const T s1 = (T(1) - L.beta) * T(0.125);
  const T ih2 = L.ih * L.ih;
  const T cn = (T(1) - L.beta) / T(6);
  cx<T> yr[3][2], yg[3][2];
  cx<T> schur = mk(L.kap[cell], T(0));
  cx<T> rp = rs[3 * L.fs + cell];
  int64_t idx[3][2];
  bool ok[3][2];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    ok[k][0] = c[k] >= 1;
    ok[k][1] = c[k] + 1 <= L.n[k] - 1;
    const T se0 = mL[k] + mc + T(0.25) * (n4[k][0] + n4[k][1]);
    const T se1 = mc + mR[k] + T(0.25) * (n4[k][1] + n4[k][2]);
    const T rf0 = T(0.5) * (rL[k] + rc), rf1 = T(0.5) * (rc + rR[k]);
    const T at = asum - acen[k];
    const cx<T> mf0 = mk(L.omega2, -L.omega2 * (L.gam + alo[k] + at));
    const cx<T> mf1 = mk(L.omega2, -L.omega2 * (L.gam + ahi[k] + at));
    cx<T> B[4];
    B[0] = ok[k][0] ? mk(s0 * ih2 * (mL[k] + mc + se0), T(0)) - (L.beta * rf0) * mf0 : mk(T(1), T(0));
    B[3] = ok[k][1] ? mk(s0 * ih2 * (mc + mR[k] + se1), T(0)) - (L.beta * rf1) * mf1 : mk(T(1), T(0));
    if (ok[k][0] && ok[k][1]) {
      B[1] = mk(-mc * s0 * ih2 + s1 * ih2 * se0, T(0)) - (cn * rf1) * mf0;
      B[2] = mk(-mc * s0 * ih2 + s1 * ih2 * se1, T(0)) - (cn * rf0) * mf1;
    } else {
      B[1] = czero<T>();
      B[2] = czero<T>();
    }
    idx[k][0] = k * L.fs + cell;
    idx[k][1] = ok[k][1] ? k * L.fs + cell + st[k] : 0;
    cx<T> g[2], d[2];
    g[0] = mk(ok[k][0] ? L.ih : T(0), T(0));
    g[1] = mk(ok[k][1] ? -L.ih : T(0), T(0));
    d[0] = mk(ok[k][0] ? -s0 * L.ih : T(0), T(0));
    d[1] = mk(ok[k][1] ? s0 * L.ih : T(0), T(0));
    if (ADJ) {  // block of H^H = conjugate transpose
      cx<T> t = B[1];
      B[0] = conj(B[0]); B[3] = conj(B[3]);
      B[1] = conj(B[2]); B[2] = conj(t);
      cx<T> g0 = g[0], g1 = g[1];
      g[0] = conj(d[0]); g[1] = conj(d[1]);
      d[0] = conj(g0); d[1] = conj(g1);
    }
    cx<T> rk[2];
    rk[0] = ok[k][0] ? rs[idx[k][0]] : czero<T>();
    rk[1] = ok[k][1] ? rs[idx[k][1]] : czero<T>();
    const cx<T> det = B[0] * B[3] - B[1] * B[2];
    const T id2 = T(1) / abs2(det);
    const cx<T> rdet = mk(det.re * id2, -det.im * id2);
    const cx<T> inv00 = B[3] * rdet, inv01 = -(B[1] * rdet), inv10 = -(B[2] * rdet), inv11 = B[0] * rdet;
    yr[k][0] = inv00 * rk[0] + inv01 * rk[1];
    yr[k][1] = inv10 * rk[0] + inv11 * rk[1];
    yg[k][0] = inv00 * g[0] + inv01 * g[1];
    yg[k][1] = inv10 * g[0] + inv11 * g[1];
    rp -= d[0] * yr[k][0] + d[1] * yr[k][1];
    schur -= d[0] * yg[k][0] + d[1] * yg[k][1];
  }
  const T is2 = T(1) / abs2(schur);
  const cx<T> dp = rp * mk(schur.re * is2, -schur.im * is2);
  if (!WR) {
    xs[3 * L.fs + cell] += w * dp;
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int sd = 0; sd < 2; ++sd)
        if (ok[k][sd]) xs[idx[k][sd]] += w * (yr[k][sd] - yg[k][sd] * dp);
    return;
  }
  const cx<T> z = czero<T>();
  xs[3 * L.fs + cell] = w * dp;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (ok[k][0]) xs[idx[k][0]] = w * (yr[k][0] - yg[k][0] * dp);
    else xs[k * L.fs + cell] = z;  // boundary face
    if (ok[k][1]) xs[idx[k][1]] = w * (yr[k][1] - yg[k][1] * dp);
  }
  if (c[0] >= 1) {
    const int64_t nb = cell - 1;
    xs[3 * L.fs + nb] = z;
    if (c[0] == 1) xs[nb] = z;
    if (c[1] == 0) xs[L.fs + nb] = z;
    if (c[2] == 0) xs[2 * L.fs + nb] = z;
  }
  if (c[0] + 1 < n0) {
    const int64_t nb = cell + 1;
    xs[3 * L.fs + nb] = z;
    if (c[1] == 0) xs[L.fs + nb] = z;
    if (c[2] == 0) xs[2 * L.fs + nb] = z;
  }
}

template <typename T>
int launch_vanka(const LevelArgs<T>& L, int dim, bool adj, const void* r, void* x, int colour, double w, int nrhs,
                 hipStream_t st, bool write) {
  if (write && dim != 3) return (int)hipErrorInvalidValue;
  const int64_t work = (L.fs / L.n[0]) * ((L.n[0] + 1) / 2);
  // small (coarse) levels: 64-thread workgroups so that every CU gets work
  const int bs = work < 256 * 256 ? 64 : 256;
  dim3 blk(bs), grd((unsigned)((work + bs - 1) / bs), nrhs);
  const cx<T>* rp = (const cx<T>*)r;
  cx<T>* xp = (cx<T>*)x;
  if (dim == 3) {
    if (work > 0x7fffffffll || L.fs > 0x7fffffffll) return (int)hipErrorInvalidValue;
    if (adj && write) ELH_LAUNCH((k_vanka3<true, true, T>), grd, blk, 0, st, L, rp, xp, colour, (T)w, nrhs);
    else if (adj) ELH_LAUNCH((k_vanka3<true, false, T>), grd, blk, 0, st, L, rp, xp, colour, (T)w, nrhs);
    else if (write) ELH_LAUNCH((k_vanka3<false, true, T>), grd, blk, 0, st, L, rp, xp, colour, (T)w, nrhs);
    else ELH_LAUNCH((k_vanka3<false, false, T>), grd, blk, 0, st, L, rp, xp, colour, (T)w, nrhs);
  } else {
    if (adj) ELH_LAUNCH((k_vanka<2, true, T>), grd, blk, 0, st, L, rp, xp, colour, (T)w, nrhs);
    else ELH_LAUNCH((k_vanka<2, false, T>), grd, blk, 0, st, L, rp, xp, colour, (T)w, nrhs);
  }
  return (int)hipGetLastError();
}
template int launch_vanka<double>(const LevelArgs<double>&, int, bool, const void*, void*, int, double, int,
                                  hipStream_t, bool);
template int launch_vanka<float>(const LevelArgs<float>&, int, bool, const void*, void*, int, double, int,
                                 hipStream_t, bool);

// ---------------------------------------------------------------------------
// MAC restriction (one thread per coarse cell) and prolongation (one thread
// per fine cell), Section 2.3
// ---------------------------------------------------------------------------
template <int DIM, typename T>
__global__ void __launch_bounds__(256) k_restrict(LevelArgs<T> F, LevelArgs<T> C, const cx<T>* __restrict__ r,
                                                   cx<T>* __restrict__ rc, int nrhs) {
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (cell >= C.fs || s >= nrhs) return;
  int c[3];
  c[0] = (int)(cell % C.n[0]);
  c[1] = (int)((cell / C.n[0]) % C.n[1]);
  c[2] = (int)(cell / ((int64_t)C.n[0] * C.n[1]));
  const cx<T>* rs = r + s * F.vs;
  cx<T>* os = rc + s * C.vs;
  const T tw = DIM == 3 ? T(0.25) : T(0.5);  // (1/2)^(d-1) transverse pair means
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    cx<T> acc = czero<T>();
    if (c[k] >= 1) {
      for (int o = -1; o <= 1; ++o) {
        const T wk = o == 0 ? T(0.5) : T(0.25);
        int nb = DIM == 3 ? 4 : 2;
        for (int b = 0; b < nb; ++b) {
          int j[3] = {2 * c[0], 2 * c[1], DIM == 3 ? 2 * c[2] : 0};
          int bit = 0;
#pragma unroll
          for (int a = 0; a < DIM; ++a) {
            if (a == k) continue;
            j[a] += (b >> bit) & 1;
            ++bit;
          }
          j[k] = 2 * c[k] + o;
          acc += (wk * tw) * rs[k * F.fs + lin<DIM>(F.n, j)];
        }
      }
    }
    os[k * C.fs + cell] = acc;
  }
  cx<T> acc = czero<T>();
  const int nch = DIM == 3 ? 8 : 4;
  for (int b = 0; b < nch; ++b) {
    int j[3] = {2 * c[0] + (b & 1), 2 * c[1] + ((b >> 1) & 1), DIM == 3 ? 2 * c[2] + ((b >> 2) & 1) : 0};
    acc += rs[DIM * F.fs + lin<DIM>(F.n, j)];
  }
  os[DIM * C.fs + cell] = (T(1) / T(nch)) * acc;
}

// Fused residual and restriction, one thread per coarse cell: rc = R (b -
// H_s x) with every fine residual row the restriction needs evaluated in
// place by the row evaluators (no fine residual is stored).  The face-normal
// full weighting makes a fine face between two coarse faces count for both,
// so about 1.4 row evaluations per fine row; this form serves the 2D and the
// small 3D levels, where launches dominate.  Weights and their order as
// k_restrict.
template <int DIM, bool ADJ, typename T>
__global__ void __launch_bounds__(256) k_restrict_resid(LevelArgs<T> F, LevelArgs<T> C, const cx<T>* __restrict__ x,
                                                         const cx<T>* __restrict__ b, cx<T>* __restrict__ rc,
                                                         int nrhs) {
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (cell >= C.fs || s >= nrhs) return;
  int c[3];
  c[0] = (int)(cell % C.n[0]);
  c[1] = (int)((cell / C.n[0]) % C.n[1]);
  c[2] = (int)(cell / ((int64_t)C.n[0] * C.n[1]));
  const cx<T>* xs = x + s * F.vs;
  const cx<T>* bs = b + s * F.vs;
  cx<T>* os = rc + s * C.vs;
  const T tw = DIM == 3 ? T(0.25) : T(0.5);
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    cx<T> acc = czero<T>();
    if (c[k] >= 1) {
      for (int o = -1; o <= 1; ++o) {
        const T wk = o == 0 ? T(0.5) : T(0.25);
        const int nb = DIM == 3 ? 4 : 2;
        for (int bb = 0; bb < nb; ++bb) {
          int j[3] = {2 * c[0], 2 * c[1], DIM == 3 ? 2 * c[2] : 0};
          int bit = 0;
#pragma unroll
          for (int a = 0; a < DIM; ++a) {
            if (a == k) continue;
            j[a] += (bb >> bit) & 1;
            ++bit;
          }
          j[k] = 2 * c[k] + o;  // >= 1: never a boundary face
          const cx<T> r = bs[k * F.fs + lin<DIM>(F.n, j)] - eval_u<DIM, ADJ>(xs, F, k, j);
          acc += (wk * tw) * r;
        }
      }
    }
    os[k * C.fs + cell] = acc;
  }
  cx<T> acc = czero<T>();
  const int nch = DIM == 3 ? 8 : 4;
  for (int bb = 0; bb < nch; ++bb) {
    int j[3] = {2 * c[0] + (bb & 1), 2 * c[1] + ((bb >> 1) & 1), DIM == 3 ? 2 * c[2] + ((bb >> 2) & 1) : 0};
    acc += bs[DIM * F.fs + lin<DIM>(F.n, j)] - eval_p<DIM, ADJ>(xs, F, j);
  }
  os[DIM * C.fs + cell] = (T(1) / T(nch)) * acc;
}

template <int DIM, typename T>
__global__ void __launch_bounds__(256) k_prolong_add(LevelArgs<T> F, LevelArgs<T> C, const cx<T>* __restrict__ e,
                                                      cx<T>* __restrict__ x, int nrhs) {
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (cell >= F.fs || s >= nrhs) return;
  int i[3];
  i[0] = (int)(cell % F.n[0]);
  i[1] = (int)((cell / F.n[0]) % F.n[1]);
  i[2] = (int)(cell / ((int64_t)F.n[0] * F.n[1]));
  const cx<T>* es = e + s * C.vs;
  cx<T>* xs = x + s * F.vs;
  // 1D interpolation stencils per axis: up to two coarse indices + weights
  for (int f = 0; f <= DIM; ++f) {
    if (f < DIM && i[f] == 0) continue;  // boundary face stays zero
    int J[3][2];
    T W[3][2];
    int cnt[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cnt[a] = 0;
      if (a >= DIM) { J[a][0] = 0; W[a][0] = T(1); cnt[a] = 1; continue; }
      if (a == f) {  // face-normal linear interpolation
        if ((i[a] & 1) == 0) {
          int jj = i[a] >> 1;
          if (jj >= 1 && jj <= C.n[a] - 1) { J[a][cnt[a]] = jj; W[a][cnt[a]] = T(1); ++cnt[a]; }
        } else {
          int j0 = (i[a] - 1) >> 1, j1 = (i[a] + 1) >> 1;
          if (j0 >= 1 && j0 <= C.n[a] - 1) { J[a][cnt[a]] = j0; W[a][cnt[a]] = T(0.5); ++cnt[a]; }
          if (j1 >= 1 && j1 <= C.n[a] - 1) { J[a][cnt[a]] = j1; W[a][cnt[a]] = T(0.5); ++cnt[a]; }
        }
      } else {  // cell linear interpolation, weights 3/4 and 1/4
        int I = i[a] >> 1;
        J[a][cnt[a]] = I; W[a][cnt[a]] = T(0.75); ++cnt[a];
        int I2 = (i[a] & 1) ? I + 1 : I - 1;
        if (I2 >= 0 && I2 <= C.n[a] - 1) { J[a][cnt[a]] = I2; W[a][cnt[a]] = T(0.25); ++cnt[a]; }
      }
    }
    cx<T> acc = czero<T>();
    for (int a0 = 0; a0 < cnt[0]; ++a0)
      for (int a1 = 0; a1 < cnt[1]; ++a1)
        for (int a2 = 0; a2 < cnt[2]; ++a2) {
          int j[3] = {J[0][a0], J[1][a1], J[2][a2]};
          acc += (W[0][a0] * W[1][a1] * W[2][a2]) * es[f * C.fs + lin<DIM>(C.n, j)];
        }
    xs[f * F.fs + cell] += acc;
  }
}

// 3D prolongation-add with fixed coarse stencils: x_2 and x_3 take two
// coarse indices (clamped to the coarse grid) and weights that are zero
// where the variable-length stencil of k_prolong_add has no term, so the
// loop nest has no data-dependent trip counts; x_1 takes the three coarse
// indices a pair of fine cells needs.  Same weights as k_prolong_add: linear
// along the face normal (coincident fine faces take the coarse face, odd
// faces the mean of the two beside them, boundary coarse faces contribute
// zero), 3/4 - 1/4 across cells.
template <typename T>
__global__ void __launch_bounds__(256) k_prolong3(LevelArgs<T> F, LevelArgs<T> C, const cx<T>* __restrict__ e,
                                                   cx<T>* __restrict__ x, int nrhs) {
  // One thread per pair of fine cells (2I, 2I+1) along x_1 (fine n_1 is
  // even on every level that prolongs): both share the coarse x_1
  // neighbourhood I-1, I, I+1.  Weights are exact dyadic fractions and the
  // terms are added in the same order as one cell at a time would.
  const int hp = F.n[0] >> 1;
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (id >= hp * F.n[1] * F.n[2] || s >= nrhs) return;
  const int I = id % hp;
  const int t = id / hp;
  int i[3];
  i[0] = 2 * I;
  i[1] = t % F.n[1];
  i[2] = t / F.n[1];
  const int cs[3] = {1, C.n[0], C.n[0] * C.n[1]};
  // axes x_2, x_3: coarse offsets and weights of the cell stencil (c) and of
  // the face-normal stencil (f)
  int oc[3][2], of[3][2];
  T wc[3][2], wf[3][2];
#pragma unroll
  for (int a = 1; a < 3; ++a) {
    const int Ia = i[a] >> 1;
    const int I2 = (i[a] & 1) ? Ia + 1 : Ia - 1;
    const bool ok2 = I2 >= 0 && I2 < C.n[a];
    oc[a][0] = Ia * cs[a];
    oc[a][1] = (ok2 ? I2 : Ia) * cs[a];
    wc[a][0] = T(0.75);
    wc[a][1] = ok2 ? T(0.25) : T(0);
    int J0, J1;
    T v0, v1;
    if ((i[a] & 1) == 0) {
      J0 = J1 = Ia;
      v0 = T(1);
      v1 = T(0);
    } else {
      J0 = Ia;
      J1 = Ia + 1;
      v0 = v1 = T(0.5);
    }
    const bool ok0 = J0 >= 1 && J0 <= C.n[a] - 1, ok1 = J1 >= 1 && J1 <= C.n[a] - 1;
    of[a][0] = min(J0, C.n[a] - 1) * cs[a];
    of[a][1] = min(J1, C.n[a] - 1) * cs[a];
    wf[a][0] = ok0 ? v0 : T(0);
    wf[a][1] = ok1 ? v1 : T(0);
  }
  // axis x_1, cell stencil: even cell 0.75 e[I] + 0.25 e[I-1], odd cell
  // 0.75 e[I] + 0.25 e[I+1]; face stencil: even face 2I takes e[I], odd face
  // 2I+1 takes (e[I] + e[I+1]) / 2 (coarse faces 0 and n_1 are not unknowns)
  const int Im = I > 0 ? I - 1 : I, Ip = I + 1 < C.n[0] ? I + 1 : I;
  const T wm = I > 0 ? T(0.25) : T(0), wp = I + 1 < C.n[0] ? T(0.25) : T(0);
  const T fe = I >= 1 ? T(1) : T(0), fo0 = I >= 1 ? T(0.5) : T(0), fo1 = I + 1 <= C.n[0] - 1 ? T(0.5) : T(0);
  const int64_t cell = ((int64_t)i[2] * F.n[1] + i[1]) * F.n[0] + i[0];
  const cx<T>* es = e + s * C.vs;
  cx<T>* xs = x + s * F.vs;
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    if ((f == 1 && i[1] == 0) || (f == 2 && i[2] == 0)) continue;  // boundary faces stay zero
    const cx<T>* ef = es + (int64_t)f * C.fs;
    cx<T> ae = czero<T>(), ao = czero<T>();
#pragma unroll
    for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
      for (int a1 = 0; a1 < 2; ++a1) {
        const int o = (f == 1 ? of[1][a1] : oc[1][a1]) + (f == 2 ? of[2][a2] : oc[2][a2]);
        const T w12 = (f == 1 ? wf[1][a1] : wc[1][a1]) * (f == 2 ? wf[2][a2] : wc[2][a2]);
        const cx<T> eI = ef[o + I], eP = ef[o + Ip];
        if (f == 0) {
          ae += (fe * w12) * eI;
          ao += (fo0 * w12) * eI;
          ao += (fo1 * w12) * eP;
        } else {
          const cx<T> eM = ef[o + Im];
          ae += (T(0.75) * w12) * eI;
          ae += (wm * w12) * eM;
          ao += (T(0.75) * w12) * eI;
          ao += (wp * w12) * eP;
        }
      }
    // cells 2I and 2I+1 are adjacent and the pair is aligned to its size
    // (even cell index, even n_1): one wide load and one wide store
    struct alignas(2 * sizeof(cx<T>)) Pair { cx<T> a, b; };
    Pair* xf = reinterpret_cast<Pair*>(xs + (int64_t)f * F.fs + cell);
    Pair v = *xf;
    if (f != 0 || I != 0) v.a += ae;  // fine face 0 along x_1 is not an unknown
    v.b += ao;
    *xf = v;
  }
}

template <typename T>
int launch_restrict(const LevelArgs<T>& F, const LevelArgs<T>& C, int dim, const void* r, void* rc, int nrhs,
                    hipStream_t st) {
  dim3 blk(256), grd((unsigned)((C.fs + 255) / 256), nrhs);
  if (dim == 3)
    ELH_LAUNCH((k_restrict<3, T>), grd, blk, 0, st, F, C, (const cx<T>*)r, (cx<T>*)rc, nrhs);
  else
    ELH_LAUNCH((k_restrict<2, T>), grd, blk, 0, st, F, C, (const cx<T>*)r, (cx<T>*)rc, nrhs);
  return (int)hipGetLastError();
}
template <typename T>
int launch_restrict_resid(const LevelArgs<T>& F, const LevelArgs<T>& C, int dim, bool adj, const void* x,
                          const void* b, void* rc, int nrhs, hipStream_t st) {
  dim3 blk(C.fs < 256 * 64 ? 64 : 256);
  dim3 grd((unsigned)((C.fs + blk.x - 1) / blk.x), nrhs);
  const cx<T>* xp = (const cx<T>*)x;
  const cx<T>* bp = (const cx<T>*)b;
  cx<T>* op = (cx<T>*)rc;
  if (dim == 3) {
    if (adj) ELH_LAUNCH((k_restrict_resid<3, true, T>), grd, blk, 0, st, F, C, xp, bp, op, nrhs);
    else ELH_LAUNCH((k_restrict_resid<3, false, T>), grd, blk, 0, st, F, C, xp, bp, op, nrhs);
  } else {
    if (adj) ELH_LAUNCH((k_restrict_resid<2, true, T>), grd, blk, 0, st, F, C, xp, bp, op, nrhs);
    else ELH_LAUNCH((k_restrict_resid<2, false, T>), grd, blk, 0, st, F, C, xp, bp, op, nrhs);
  }
  return (int)hipGetLastError();
}
template int launch_restrict_resid<double>(const LevelArgs<double>&, const LevelArgs<double>&, int, bool,
                                           const void*, const void*, void*, int, hipStream_t);
template int launch_restrict_resid<float>(const LevelArgs<float>&, const LevelArgs<float>&, int, bool, const void*,
                                          const void*, void*, int, hipStream_t);

template <typename T>
int launch_prolong_add(const LevelArgs<T>& F, const LevelArgs<T>& C, int dim, const void* e, void* x, int nrhs,
                       hipStream_t st) {
  dim3 blk(256), grd((unsigned)((F.fs + 255) / 256), nrhs);
  // the pair kernel updates two adjacent fine cells with one aligned access
  const bool pair_aligned = reinterpret_cast<uintptr_t>(x) % (2 * sizeof(cx<T>)) == 0;
  if (dim == 3 && F.fs <= 0x7fffffffll && (F.n[0] & 1) == 0 && F.n[0] == 2 * C.n[0] && pair_aligned)
    ELH_LAUNCH((k_prolong3<T>), dim3((unsigned)((F.fs / 2 + 255) / 256), nrhs), blk, 0, st, F, C,
                       (const cx<T>*)e, (cx<T>*)x, nrhs);
  else if (dim == 3)
    ELH_LAUNCH((k_prolong_add<3, T>), grd, blk, 0, st, F, C, (const cx<T>*)e, (cx<T>*)x, nrhs);
  else
    ELH_LAUNCH((k_prolong_add<2, T>), grd, blk, 0, st, F, C, (const cx<T>*)e, (cx<T>*)x, nrhs);
  return (int)hipGetLastError();
}
template int launch_restrict<double>(const LevelArgs<double>&, const LevelArgs<double>&, int, const void*, void*,
                                     int, hipStream_t);
template int launch_restrict<float>(const LevelArgs<float>&, const LevelArgs<float>&, int, const void*, void*, int,
                                    hipStream_t);
template int launch_prolong_add<double>(const LevelArgs<double>&, const LevelArgs<double>&, int, const void*,
                                        void*, int, hipStream_t);
template int launch_prolong_add<float>(const LevelArgs<float>&, const LevelArgs<float>&, int, const void*, void*,
                                       int, hipStream_t);

// ---------------------------------------------------------------------------
// parameter gradient  g_m(c) = - Re sum_s v_s^H (dH/dm_c) u_s  (float64)
// ---------------------------------------------------------------------------
// Gather form, one thread per cell, loop over sources.  H depends on
//  * mu through A_e(mu): the x_k-derivative flux of u_k at cell c uses mu_c;
//    a transverse flux on an edge uses the mean of the four cells around it
//    (media clamped at the boundary, so a boundary edge counts a cell twice);
//  * lam and mu through kappa = 1/(lam+mu): dkappa = -kappa^2;
//  * rho through A_f(rho): the mean of the two cells beside a face.
// For the Laplacian term the derivative of v_k^H D^T diag(mu_e) D Y u_k is
// conj(D v_k) (D Y u_k) at the flux point; for the mass term
// - v_k^H diag(w2) S diag(rho_f) u_k it is - conj(S conj(w2) v_k) u_k at the face.
template <int DIM>
__global__ void __launch_bounds__(256) k_gradient(LevelArgs<double> L, int nrhs, const cx<double>* __restrict__ u,
                                                   const cx<double>* __restrict__ v, double* __restrict__ g_lam,
                                                   double* __restrict__ g_mu, double* __restrict__ g_rho) {
  typedef double T;
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= L.fs) return;
  int c[3];
  c[0] = (int)(cell % L.n[0]);
  c[1] = (int)((cell / L.n[0]) % L.n[1]);
  c[2] = (int)(cell / ((int64_t)L.n[0] * L.n[1]));
  const T kap = L.kap[cell];
  const T cn = (T(1) - L.beta) / T(2 * DIM);
  T gl = 0, gm = 0, gr = 0;
  for (int s = 0; s < nrhs; ++s) {
    const cx<T>* us = u + (int64_t)s * L.vs;
    const cx<T>* vs = v + (int64_t)s * L.vs;
    const cx<T> up = us[DIM * L.fs + cell], vp = vs[DIM * L.fs + cell];
    const T kp = kap * kap * (vp.re * up.re + vp.im * up.im);
    gl += kp;
    gm += kp;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      // flux of u_k along x_k at cell c
      {
        int j[3] = {c[0], c[1], c[2]};
        j[k] = c[k] + 1;
        cx<T> dv = ldf<DIM>(vs, L, k, j);
        j[k] = c[k];
        dv = L.ih * (dv - ldf<DIM>(vs, L, k, j));
        cx<T> dy = spread_flux<DIM>(us, L, k, k, c[k], c);
        gm -= dv.re * dy.re + dv.im * dy.im;
      }
      // transverse fluxes on the edges around cell c
#pragma unroll
      for (int l = 0; l < DIM; ++l) {
        if (l == k) continue;
        for (int f = c[k]; f <= c[k] + 1; ++f) {
          if (f < 1 || f > L.n[k] - 1) continue;
          for (int e = c[l]; e <= c[l] + 1; ++e) {
            // edge (k-face f, l-face e): cells clamp(e-1), clamp(e) along l
            T wgt = T(0.25);
            if (e == c[l] && e - 1 < 0) wgt += T(0.25);
            if (e == c[l] + 1 && e > L.n[l] - 1) wgt += T(0.25);
            int t[3] = {c[0], c[1], c[2]};
            t[k] = f;
            int j[3] = {t[0], t[1], t[2]};
            j[l] = e;
            cx<T> dv = ldf<DIM>(vs, L, k, j);
            j[l] = e - 1;
            dv = L.ih * (dv - ldf<DIM>(vs, L, k, j));
            cx<T> dy = spread_flux<DIM>(us, L, k, l, e, t);
            gm -= wgt * (dv.re * dy.re + dv.im * dy.im);
          }
        }
      }
      // spread mass on the two faces of cell c normal to x_k
      for (int f = c[k]; f <= c[k] + 1; ++f) {
        if (f < 1 || f > L.n[k] - 1) continue;
        int F[3] = {c[0], c[1], c[2]};
        F[k] = f;
        cx<T> w = L.beta * (conj(mass_factor<DIM>(L, k, F)) * vs[k * L.fs + lin<DIM>(L.n, F)]);
#pragma unroll
        for (int a = 0; a < DIM; ++a)
#pragma unroll
          for (int sg = -1; sg <= 1; sg += 2) {
            int Q[3] = {F[0], F[1], F[2]};
            Q[a] += sg;
            if (!in_grid<DIM>(L.n, Q) || Q[k] == 0) continue;
            w += cn * (conj(mass_factor<DIM>(L, k, Q)) * vs[k * L.fs + lin<DIM>(L.n, Q)]);
          }
        const cx<T> uf = us[k * L.fs + lin<DIM>(L.n, F)];
        gr += T(0.5) * (w.re * uf.re + w.im * uf.im);
      }
    }
  }
  g_lam[cell] = gl;
  g_mu[cell] = gm;
  g_rho[cell] = gr;
}

int launch_gradient(const LevelArgs<double>& L, int dim, int nrhs, const void* u, const void* v, double* gl,
                    double* gm, double* gr, hipStream_t st) {
  dim3 blk(256), grd((unsigned)((L.fs + 255) / 256));
  if (dim == 3)
    ELH_LAUNCH(k_gradient<3>, grd, blk, 0, st, L, nrhs, (const cx<double>*)u, (const cx<double>*)v, gl, gm, gr);
  else
    ELH_LAUNCH(k_gradient<2>, grd, blk, 0, st, L, nrhs, (const cx<double>*)u, (const cx<double>*)v, gl, gm, gr);
  return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// media setup: child means, kappa, casts
// ---------------------------------------------------------------------------
__global__ void k_coarsen_media(int dim, int f0, int f1, int f2, const double* __restrict__ a, double* __restrict__ out) {
  const int c0 = f0 / 2, c1 = f1 / 2, c2 = dim == 3 ? f2 / 2 : 1;
  const int64_t n = (int64_t)c0 * c1 * c2;
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= n) return;
  int i0 = (int)(cell % c0), i1 = (int)((cell / c0) % c1), i2 = (int)(cell / ((int64_t)c0 * c1));
  double s = 0.0;
  const int nz = dim == 3 ? 2 : 1;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < 2; ++y)
      for (int xx = 0; xx < 2; ++xx) {
        int64_t j = ((int64_t)(dim == 3 ? 2 * i2 + z : 0) * f1 + (2 * i1 + y)) * f0 + (2 * i0 + xx);
        s += a[j];
      }
  // mean of the 2^d children, summed in the order x1 pairs, then x2, x3
  out[cell] = s / (double)(dim == 3 ? 8 : 4);
}

__global__ void k_media_finish(int64_t n, const double* __restrict__ lam, const double* __restrict__ mu,
                               const double* __restrict__ rho, double* __restrict__ kap, float* __restrict__ mu32,
                               float* __restrict__ rho32, float* __restrict__ kap32) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double k = 1.0 / (lam[i] + mu[i]);
  kap[i] = k;
  mu32[i] = (float)mu[i];
  rho32[i] = (float)rho[i];
  kap32[i] = (float)k;
}

int launch_coarsen_media(int dim, const int* nf, const double* a, double* out, hipStream_t st) {
  int64_t n = (int64_t)(nf[0] / 2) * (nf[1] / 2) * (dim == 3 ? nf[2] / 2 : 1);
  ELH_LAUNCH(k_coarsen_media, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dim, nf[0], nf[1],
                     nf[2], a, out);
  return (int)hipGetLastError();
}
int launch_media_finish(int64_t n, const double* lam, const double* mu, const double* rho, double* kap, float* mu32,
                        float* rho32, float* kap32, hipStream_t st) {
  ELH_LAUNCH(k_media_finish, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, lam, mu, rho, kap,
                     mu32, rho32, kap32);
  return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Krylov vector operations on batches of complex vectors (nrhs x len).
// Reductions accumulate in float64, two stages, fixed order.
// ---------------------------------------------------------------------------
// The partial-sum scratch holds RED_PAIRS (block, entry) pairs per rhs
// (512 * MAXDOT): a reduction over m entries may use up to RED_PAIRS / m
// blocks, enough to keep every CU streaming on the large vectors.
constexpr int RED_PAIRS = 512 * MAXDOT;
constexpr int RED_THREADS = 256;

// MC > 0: exactly MC dots (accumulators and loop fixed at compile time);
// MC = 0: m dots, m <= MAXDOT.
template <typename TV, typename TW, int MC>
__global__ void __launch_bounds__(RED_THREADS) k_multidot(int m, const TV* __restrict__ V, int64_t vstride_vec,
                                                           int64_t vstride_rhs, const TW* __restrict__ w,
                                                           int64_t wstride_rhs, int64_t len,
                                                           double* __restrict__ part) {
  // part[(s*gridDim.x + block)*m*2 + 2i (+1)] = partial of <V_i, w>
  constexpr int NA = MC > 0 ? MC : MAXDOT;
  if (MC > 0) m = MC;
  const int s = blockIdx.y;
  double acc_re[NA], acc_im[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) { acc_re[i] = 0; acc_im[i] = 0; }
  const TW* ws = w + s * wstride_rhs;
  const TV* vs = V + s * vstride_rhs;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < len; t += (int64_t)gridDim.x * blockDim.x) {
    auto wv = ws[t];
    double wr = (double)wv.re, wi = (double)wv.im;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      if (MC > 0 || i < m) {
        auto vv = vs[i * vstride_vec + t];
        double vr = (double)vv.re, vi = (double)vv.im;
        acc_re[i] += vr * wr + vi * wi;  // conj(v) * w
        acc_im[i] += vr * wi - vi * wr;
      }
    }
  }
  __shared__ double red[RED_THREADS];
  for (int i = 0; i < m; ++i) {
    for (int part_ri = 0; part_ri < 2; ++part_ri) {
      double v = 0;
#pragma unroll
      for (int k = 0; k < NA; ++k)
        if (k == i) v = part_ri == 0 ? acc_re[k] : acc_im[k];
      red[threadIdx.x] = v;
      __syncthreads();
      for (int o = RED_THREADS / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
      }
      if (threadIdx.x == 0) part[((int64_t)s * gridDim.x + blockIdx.x) * m * 2 + 2 * i + part_ri] = red[0];
      __syncthreads();
    }
  }
}

__global__ void __launch_bounds__(256) k_reduce_parts(int m2, int nblocks, const double* __restrict__ part,
                                                      double* __restrict__ out) {
  // one workgroup per (entry, rhs): strided partial sums, then a fixed tree
  const int e = blockIdx.x, s = blockIdx.y;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) acc += part[((int64_t)s * nblocks + b) * m2 + e];
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[(int64_t)s * m2 + e] = red[0];
}

int multidot_blocks(int m, int64_t len, int cap) {
  int64_t nb = (len + RED_THREADS - 1) / RED_THREADS;
  if (nb > RED_PAIRS / m) nb = RED_PAIRS / m;
  if (nb > cap) nb = cap;
  return nb < 1 ? 1 : (int)nb;
}
int norm_blocks(int64_t len, int cap) {
  int64_t nb = (len + RED_THREADS - 1) / RED_THREADS;
  if (nb > RED_PAIRS) nb = RED_PAIRS;
  if (nb > cap) nb = cap;
  return nb < 1 ? 1 : (int)nb;
}

// The consumers of a small reduction (GMRES bookkeeping, K-cycle
// coefficients: at most FUSE_VALS values, whose producers were launched with
// at most FUSE_BLOCKS blocks) finish it themselves, which saves one launch
// per reduction.  The block of 256 threads splits into one group per value
// (a power of two of threads each); a group sums its value's partials
// strided, then a fixed tree inside the group.  Otherwise `out` holds the
// values reduced by k_reduce_parts.  Every thread of the block must call
// this before any early return.
__device__ const double* small_reduction(int nv, int m2, const double* __restrict__ out,
                                         const double* __restrict__ part, int nb, double* vals) {
  if (!part) return out;
  __shared__ double red[256];
  int gs = 256;  // threads per value
  while (gs > 16 && 256 / gs < nv) gs >>= 1;
  const int v = threadIdx.x / gs, lane = threadIdx.x - v * gs;
  double acc = 0.0;
  if (v < nv) {
    const int sv = v / m2, e = v - sv * m2;
    for (int b = lane; b < nb; b += gs) acc += part[((int64_t)sv * nb + b) * m2 + e];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = gs / 2; o > 0; o >>= 1) {
    if (lane < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (v < nv && lane == 0) vals[v] = red[threadIdx.x];
  __syncthreads();
  return vals;
}

template <typename TV, typename TW>
int launch_multidot(int m, const void* V, int64_t vstride_vec, int64_t vstride_rhs, const void* w,
                    int64_t wstride_rhs, int64_t len, int nrhs, double* part, double* out, hipStream_t st) {
  if (m < 1 || m > MAXDOT) return (int)hipErrorInvalidValue;
  const int nb = multidot_blocks(m, len, out ? RED_PAIRS : FUSE_BLOCKS);
  const dim3 grd(nb, nrhs), blk(RED_THREADS);
  const TV* Vp = (const TV*)V;
  const TW* wp = (const TW*)w;
  switch (m) {
    case 1: ELH_LAUNCH((k_multidot<TV, TW, 1>), grd, blk, 0, st, m, Vp, vstride_vec, vstride_rhs, wp, wstride_rhs, len, part); break;
    case 2: ELH_LAUNCH((k_multidot<TV, TW, 2>), grd, blk, 0, st, m, Vp, vstride_vec, vstride_rhs, wp, wstride_rhs, len, part); break;
    case 3: ELH_LAUNCH((k_multidot<TV, TW, 3>), grd, blk, 0, st, m, Vp, vstride_vec, vstride_rhs, wp, wstride_rhs, len, part); break;
    case 4: ELH_LAUNCH((k_multidot<TV, TW, 4>), grd, blk, 0, st, m, Vp, vstride_vec, vstride_rhs, wp, wstride_rhs, len, part); break;
    case 5: ELH_LAUNCH((k_multidot<TV, TW, 5>), grd, blk, 0, st, m, Vp, vstride_vec, vstride_rhs, wp, wstride_rhs, len, part); break;
    case 6: ELH_LAUNCH((k_multidot<TV, TW, 6>), grd, blk, 0, st, m, Vp, vstride_vec, vstride_rhs, wp, wstride_rhs, len, part); break;
    default: ELH_LAUNCH((k_multidot<TV, TW, 0>), grd, blk, 0, st, m, Vp, vstride_vec, vstride_rhs, wp, wstride_rhs, len, part);
  }
  if (out) ELH_LAUNCH(k_reduce_parts, dim3(2 * m, nrhs), dim3(256), 0, st, 2 * m, nb, part, out);
  return (int)hipGetLastError();
}
template int launch_multidot<cx<double>, cx<double>>(int, const void*, int64_t, int64_t, const void*, int64_t,
                                                     int64_t, int, double*, double*, hipStream_t);
template int launch_multidot<cx<float>, cx<float>>(int, const void*, int64_t, int64_t, const void*, int64_t,
                                                   int64_t, int, double*, double*, hipStream_t);

// w[s] += sum_i coef[s*m+i] * V_i[s]   (coef complex double, on device);
// SET: w[s] = sum_i ... (w is not read)
template <typename TV, typename TW, bool SET>
__global__ void __launch_bounds__(256) k_multiaxpy(int m, const double* __restrict__ coef, const TV* __restrict__ V,
                                                    int64_t vstride_vec, int64_t vstride_rhs, TW* __restrict__ w,
                                                    int64_t wstride_rhs, int64_t len) {
  const int s = blockIdx.y;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= len) return;
  TW wv;
  if (!SET) wv = w[s * wstride_rhs + t];
  double re = SET ? 0.0 : (double)wv.re, im = SET ? 0.0 : (double)wv.im;
  for (int i = 0; i < m; ++i) {
    double cr = coef[(s * m + i) * 2], ci = coef[(s * m + i) * 2 + 1];
    auto vv = V[i * vstride_vec + s * vstride_rhs + t];
    double vr = (double)vv.re, vi = (double)vv.im;
    re += cr * vr - ci * vi;
    im += cr * vi + ci * vr;
  }
  wv.re = re;
  wv.im = im;
  w[s * wstride_rhs + t] = wv;
}

template <typename TV, typename TW>
int launch_multiaxpy(int m, const double* coef, const void* V, int64_t vstride_vec, int64_t vstride_rhs, void* w,
                     int64_t wstride_rhs, int64_t len, int nrhs, hipStream_t st, bool set) {
  const dim3 grd((unsigned)((len + 255) / 256), nrhs), blk(256);
  if (set)
    ELH_LAUNCH((k_multiaxpy<TV, TW, true>), grd, blk, 0, st, m, coef, (const TV*)V, vstride_vec, vstride_rhs,
                       (TW*)w, wstride_rhs, len);
  else
    ELH_LAUNCH((k_multiaxpy<TV, TW, false>), grd, blk, 0, st, m, coef, (const TV*)V, vstride_vec,
                       vstride_rhs, (TW*)w, wstride_rhs, len);
  return (int)hipGetLastError();
}
template int launch_multiaxpy<cx<double>, cx<double>>(int, const double*, const void*, int64_t, int64_t, void*,
                                                      int64_t, int64_t, int, hipStream_t, bool);
template int launch_multiaxpy<cx<float>, cx<double>>(int, const double*, const void*, int64_t, int64_t, void*,
                                                     int64_t, int64_t, int, hipStream_t, bool);
template int launch_multiaxpy<cx<float>, cx<float>>(int, const double*, const void*, int64_t, int64_t, void*,
                                                    int64_t, int64_t, int, hipStream_t, bool);

// Gram-Schmidt update fused with its norm: w[s] += sum_i coef[s*m+i] V_i[s]
// in place, part[] receives per-block partial sums of |w|^2 (entries 2b and
// 2b+1, the second zero, so k_reduce_parts yields ||w||^2 as a complex
// number), and when f is non-NULL the updated w is also written to f in
// precision TF (the input of the next preconditioner application).
template <typename TV, typename TF, int MC>
__global__ void __launch_bounds__(RED_THREADS) k_axpy_norm(int m, const double* __restrict__ coef,
                                                            const TV* __restrict__ V, int64_t vstride_vec,
                                                            int64_t vstride_rhs, TV* __restrict__ w,
                                                            int64_t wstride_rhs, TF* __restrict__ f,
                                                            int64_t fstride_rhs, int64_t len,
                                                            double* __restrict__ part) {
  constexpr int NA = MC > 0 ? MC : MAXDOT;
  if (MC > 0) m = MC;
  const int s = blockIdx.y;
  double cr[NA], ci[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    cr[i] = i < m ? coef[(s * m + i) * 2] : 0.0;
    ci[i] = i < m ? coef[(s * m + i) * 2 + 1] : 0.0;
  }
  double acc = 0.0;
  TV* ws = w + s * wstride_rhs;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < len; t += (int64_t)gridDim.x * blockDim.x) {
    auto wv = ws[t];
    double re = (double)wv.re, im = (double)wv.im;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      if (MC > 0 || i < m) {
        auto vv = V[i * vstride_vec + s * vstride_rhs + t];
        const double vr = (double)vv.re, vi = (double)vv.im;
        re += cr[i] * vr - ci[i] * vi;
        im += cr[i] * vi + ci[i] * vr;
      }
    }
    wv.re = re;
    wv.im = im;
    ws[t] = wv;
    if (f) {
      TF fv;
      fv.re = re;
      fv.im = im;
      f[s * fstride_rhs + t] = fv;
    }
    acc += re * re + im * im;
  }
  __shared__ double red[RED_THREADS];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = RED_THREADS / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[((int64_t)s * gridDim.x + blockIdx.x) * 2] = red[0];
    part[((int64_t)s * gridDim.x + blockIdx.x) * 2 + 1] = 0.0;
  }
}

template <typename TV, typename TF>
int launch_axpy_norm(int m, const double* coef, const void* V, int64_t vstride_vec, int64_t vstride_rhs, void* w,
                     int64_t wstride_rhs, void* f, int64_t fstride_rhs, int64_t len, int nrhs, double* part,
                     double* out, hipStream_t st) {
  if (m > MAXDOT) return (int)hipErrorInvalidValue;
  const int nb = norm_blocks(len, out ? RED_PAIRS : FUSE_BLOCKS);
  const dim3 grd(nb, nrhs), blk(RED_THREADS);
  const TV* Vp = (const TV*)V;
  switch (m) {
    case 1: ELH_LAUNCH((k_axpy_norm<TV, TF, 1>), grd, blk, 0, st, m, coef, Vp, vstride_vec, vstride_rhs, (TV*)w, wstride_rhs, (TF*)f, fstride_rhs, len, part); break;
    case 2: ELH_LAUNCH((k_axpy_norm<TV, TF, 2>), grd, blk, 0, st, m, coef, Vp, vstride_vec, vstride_rhs, (TV*)w, wstride_rhs, (TF*)f, fstride_rhs, len, part); break;
    case 3: ELH_LAUNCH((k_axpy_norm<TV, TF, 3>), grd, blk, 0, st, m, coef, Vp, vstride_vec, vstride_rhs, (TV*)w, wstride_rhs, (TF*)f, fstride_rhs, len, part); break;
    case 4: ELH_LAUNCH((k_axpy_norm<TV, TF, 4>), grd, blk, 0, st, m, coef, Vp, vstride_vec, vstride_rhs, (TV*)w, wstride_rhs, (TF*)f, fstride_rhs, len, part); break;
    case 5: ELH_LAUNCH((k_axpy_norm<TV, TF, 5>), grd, blk, 0, st, m, coef, Vp, vstride_vec, vstride_rhs, (TV*)w, wstride_rhs, (TF*)f, fstride_rhs, len, part); break;
    default: ELH_LAUNCH((k_axpy_norm<TV, TF, 0>), grd, blk, 0, st, m, coef, Vp, vstride_vec, vstride_rhs, (TV*)w, wstride_rhs, (TF*)f, fstride_rhs, len, part);
  }
  if (out) ELH_LAUNCH(k_reduce_parts, dim3(2, nrhs), dim3(256), 0, st, 2, nb, part, out);
  return (int)hipGetLastError();
}
template int launch_axpy_norm<cx<double>, cx<float>>(int, const double*, const void*, int64_t, int64_t, void*,
                                                     int64_t, void*, int64_t, int64_t, int, double*, double*,
                                                     hipStream_t);
template int launch_axpy_norm<cx<double>, cx<double>>(int, const double*, const void*, int64_t, int64_t, void*,
                                                      int64_t, void*, int64_t, int64_t, int, double*, double*,
                                                      hipStream_t);
template int launch_axpy_norm<cx<float>, cx<float>>(int, const double*, const void*, int64_t, int64_t, void*,
                                                    int64_t, void*, int64_t, int64_t, int, double*, double*,
                                                    hipStream_t);

// K-cycle coefficients, one thread per rhs (dots from k_multidot: entry i
// of rhs s at dots[(s*m + i)*2], complex).
// stage 1: dots = <V1,V1>, <R1,V1>          (m = 2)
//   a1 = conj(<R1,V1>) / <V1,V1>;  coef[s] = -a1 (for R1 += coef V1);
//   state[s] = (a1, <V1,V1>).
// stage 2: dots = <V1,V2>, <R1,V2>, <V2,V2> (m = 3), R1 now r1 = rc - a1 V1
//   b = <V1,V2>/<V1,V1>,  n2 = <V2,V2> - |<V1,V2>|^2/<V1,V1>  (= |V2 - b V1|^2),
//   a2 = conj(<R1,V2>)/n2  (<V2 - b V1, r1> = <V2, r1> since r1 is orthogonal to V1),
//   coef[s] = (a1 - a2 b, a2)  for  e = coef0 E1 + coef1 E2.
// Zero denominators give zero coefficients.
__global__ void __launch_bounds__(256) k_kcycle_coef(int stage, const double* __restrict__ dots_in,
                                                      const double* __restrict__ part, int nb,
                                                      double* __restrict__ coef, double* __restrict__ state,
                                                      int nrhs) {
  __shared__ double vals[FUSE_VALS];
  const int m2 = stage == 1 ? 4 : 6;
  const double* __restrict__ dots = small_reduction(nrhs * m2, m2, dots_in, part, nb, vals);
  const int s = threadIdx.x;
  if (s >= nrhs) return;
  if (stage == 1) {
    const double d11 = dots[(s * 2 + 0) * 2];
    const double rr = dots[(s * 2 + 1) * 2], ri = dots[(s * 2 + 1) * 2 + 1];
    const double a1r = d11 != 0.0 ? rr / d11 : 0.0, a1i = d11 != 0.0 ? -ri / d11 : 0.0;
    coef[s * 2] = -a1r;
    coef[s * 2 + 1] = -a1i;
    state[s * 4] = a1r;
    state[s * 4 + 1] = a1i;
    state[s * 4 + 2] = d11;
    state[s * 4 + 3] = 0.0;
  } else {
    const double a1r = state[s * 4], a1i = state[s * 4 + 1], d11 = state[s * 4 + 2];
    const double pr = dots[(s * 3 + 0) * 2], pi = dots[(s * 3 + 0) * 2 + 1];   // <V1,V2>
    const double qr = dots[(s * 3 + 1) * 2], qi = dots[(s * 3 + 1) * 2 + 1];   // <R1,V2>
    const double d22 = dots[(s * 3 + 2) * 2];                                   // <V2,V2>
    const double br = d11 != 0.0 ? pr / d11 : 0.0, bi = d11 != 0.0 ? pi / d11 : 0.0;
    const double n2 = d11 != 0.0 ? d22 - (pr * pr + pi * pi) / d11 : d22;
    const double a2r = n2 > 0.0 ? qr / n2 : 0.0, a2i = n2 > 0.0 ? -qi / n2 : 0.0;
    coef[s * 4] = a1r - (a2r * br - a2i * bi);
    coef[s * 4 + 1] = a1i - (a2r * bi + a2i * br);
    coef[s * 4 + 2] = a2r;
    coef[s * 4 + 3] = a2i;
  }
}

int launch_kcycle_coef(int stage, const double* dots, const double* part, int nb, double* coef, double* state,
                       int nrhs, hipStream_t st) {
  if (nrhs < 1 || nrhs > MAXRHS_KRYLOV || (part && nrhs * (stage == 1 ? 4 : 6) > FUSE_VALS))
    return (int)hipErrorInvalidValue;
  ELH_LAUNCH(k_kcycle_coef, dim3(1), dim3(256), 0, st, stage, dots, part, nb, coef, state, nrhs);
  return (int)hipGetLastError();
}

// y[s] = a[s] * x[s]   (a complex double per rhs), with type conversion
template <typename TX, typename TY>
__global__ void __launch_bounds__(256) k_scale_copy(const double* __restrict__ a, const TX* __restrict__ x,
                                                     int64_t xstride, TY* __restrict__ y, int64_t ystride,
                                                     int64_t len) {
  const int s = blockIdx.y;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= len) return;
  double ar = a ? a[2 * s] : 1.0, ai = a ? a[2 * s + 1] : 0.0;
  auto xv = x[s * xstride + t];
  double xr = (double)xv.re, xi = (double)xv.im;
  TY out;
  out.re = ar * xr - ai * xi;
  out.im = ar * xi + ai * xr;
  y[s * ystride + t] = out;
}

template <typename TX, typename TY>
int launch_scale_copy(const double* a, const void* x, int64_t xstride, void* y, int64_t ystride, int64_t len,
                      int nrhs, hipStream_t st) {
  ELH_LAUNCH((k_scale_copy<TX, TY>), dim3((unsigned)((len + 255) / 256), nrhs), dim3(256), 0, st, a,
                     (const TX*)x, xstride, (TY*)y, ystride, len);
  return (int)hipGetLastError();
}
template int launch_scale_copy<cx<double>, cx<double>>(const double*, const void*, int64_t, void*, int64_t, int64_t,
                                                       int, hipStream_t);
template int launch_scale_copy<cx<double>, cx<float>>(const double*, const void*, int64_t, void*, int64_t, int64_t,
                                                      int, hipStream_t);
template int launch_scale_copy<cx<float>, cx<double>>(const double*, const void*, int64_t, void*, int64_t, int64_t,
                                                      int, hipStream_t);
template int launch_scale_copy<cx<float>, cx<float>>(const double*, const void*, int64_t, void*, int64_t, int64_t,
                                                     int, hipStream_t);

// ---------------------------------------------------------------------------
// Device-resident GMRES bookkeeping (one thread per right-hand side): the
// Hessenberg column, complex Givens rotations, the residual estimate and the
// least-squares back substitution stay on the GPU, so a fixed-budget solve
// needs no host round trip (and can be captured in a graph).
// State layout per rhs s (doubles): see GmresDev in elh_internal.h.
// ---------------------------------------------------------------------------
struct zc { double re, im; };
__device__ inline zc zmul(zc a, zc b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline zc zconj(zc a) { return {a.re, -a.im}; }
__device__ inline double zabs(zc a) { return hypot(a.re, a.im); }

__device__ inline zc* gm_H(double* st, int s, int i, int j) {  // H[i][j], i < MAXDOT, j < MAXDOT
  return (zc*)(st + (size_t)s * GM_STRIDE) + i * MAXDOT + j;
}
__device__ inline zc* gm_g(double* st, int s) { return (zc*)(st + (size_t)s * GM_STRIDE + 2 * MAXDOT * MAXDOT); }
__device__ inline zc* gm_sn(double* st, int s) { return gm_g(st, s) + MAXDOT; }
__device__ inline double* gm_cs(double* st, int s) { return (double*)(gm_sn(st, s) + MAXDOT); }

// start of a restart cycle: beta = ||r||, g = (beta, 0, ...), scale = 1/beta
// restart start for rhs s: g = ||r0|| e_1, scale = 1/||r0||
__device__ void gm_start_rhs(int s, const double* __restrict__ nrm2, double* __restrict__ st,
                             double* __restrict__ scale) {
  double beta = sqrt(nrm2[2 * s]);
  zc* g = gm_g(st, s);
  for (int i = 0; i < MAXDOT; ++i) g[i] = {0.0, 0.0};
  g[0] = {beta, 0.0};
  scale[2 * s] = beta > 0 ? 1.0 / beta : 0.0;
  scale[2 * s + 1] = 0.0;
}

__global__ void __launch_bounds__(256) k_gm_start(int nrhs, const double* __restrict__ nrm2_in,
                                                   const double* __restrict__ part, int nb,
                                                   double* __restrict__ st, double* __restrict__ scale) {
  __shared__ double vals[FUSE_VALS];
  const double* __restrict__ nrm2 = small_reduction(nrhs * 2, 2, nrm2_in, part, nb, vals);
  int s = threadIdx.x;
  if (s >= nrhs) return;
  gm_start_rhs(s, nrm2, st, scale);
}

// after the dots h_i = <V_i, w>, i <= j: store column j and coef = -h
__global__ void __launch_bounds__(256) k_gm_hcol(int nrhs, int j, const double* __restrict__ dots_in,
                                                  const double* __restrict__ part, int nb,
                                                  double* __restrict__ st, double* __restrict__ coef) {
  __shared__ double vals[FUSE_VALS];
  const double* __restrict__ dots = small_reduction(nrhs * 2 * (j + 1), 2 * (j + 1), dots_in, part, nb, vals);
  int s = threadIdx.x;
  if (s >= nrhs) return;
  for (int i = 0; i <= j; ++i) {
    zc h = {dots[(s * (j + 1) + i) * 2], dots[(s * (j + 1) + i) * 2 + 1]};
    *gm_H(st, s, i, j) = h;
    coef[(s * (j + 1) + i) * 2] = -h.re;
    coef[(s * (j + 1) + i) * 2 + 1] = -h.im;
  }
}

// after ||w||^2, for rhs s: subdiagonal, previous rotations, new rotation,
// g update, scale = 1/h_{j+1,j}
__device__ void gm_rotate_rhs(int s, int j, const double* __restrict__ nrm2, double* __restrict__ st,
                              double* __restrict__ scale) {
  double hn = sqrt(nrm2[2 * s]);
  *gm_H(st, s, j + 1, j) = {hn, 0.0};
  zc* sn = gm_sn(st, s);
  double* cs = gm_cs(st, s);
  for (int i = 0; i < j; ++i) {
    zc a = *gm_H(st, s, i, j), b = *gm_H(st, s, i + 1, j);
    zc t = zmul(sn[i], b);
    zc na = {cs[i] * a.re + t.re, cs[i] * a.im + t.im};
    zc u = zmul(zconj(sn[i]), a);
    zc nb = {-u.re + cs[i] * b.re, -u.im + cs[i] * b.im};
    *gm_H(st, s, i, j) = na;
    *gm_H(st, s, i + 1, j) = nb;
  }
  zc a = *gm_H(st, s, j, j), b = *gm_H(st, s, j + 1, j);
  double c;
  zc sg;
  double aa = zabs(a), bb = zabs(b);
  if (bb == 0) { c = 1; sg = {0, 0}; }
  else if (aa == 0) { c = 0; sg = {b.re / bb, -b.im / bb}; }
  else {
    double den = hypot(aa, bb);
    c = aa / den;
    zc ph = {a.re / aa, a.im / aa};
    sg = zmul(ph, zc{b.re / den, -b.im / den});
  }
  cs[j] = c;
  sn[j] = sg;
  zc t = zmul(sg, b);
  *gm_H(st, s, j, j) = {c * a.re + t.re, c * a.im + t.im};
  *gm_H(st, s, j + 1, j) = {0, 0};
  zc* g = gm_g(st, s);
  zc gj = g[j];
  zc u = zmul(zconj(sg), gj);
  g[j + 1] = {-u.re, -u.im};
  g[j] = {c * gj.re, c * gj.im};
  scale[2 * s] = hn > 0 ? 1.0 / hn : 0.0;
  scale[2 * s + 1] = 0.0;
}

// y = R^{-1} g over k columns for rhs s (zero where the triangle is singular)
__device__ void gm_backsolve_rhs(int s, int k, const double* __restrict__ st, double* __restrict__ coef) {
  double* stw = const_cast<double*>(st);
  const zc* g = gm_g(stw, s);
  zc y[MAXDOT];
  for (int i = k - 1; i >= 0; --i) {
    zc acc = g[i];
    for (int q = i + 1; q < k; ++q) {
      zc t = zmul(*gm_H(stw, s, i, q), y[q]);
      acc.re -= t.re;
      acc.im -= t.im;
    }
    zc d = *gm_H(stw, s, i, i);
    double dd = d.re * d.re + d.im * d.im;
    y[i] = dd > 0 ? zc{(acc.re * d.re + acc.im * d.im) / dd, (acc.im * d.re - acc.re * d.im) / dd} : zc{0, 0};
  }
  for (int i = 0; i < k; ++i) {
    coef[(s * k + i) * 2] = y[i].re;
    coef[(s * k + i) * 2 + 1] = y[i].im;
  }
}

// bk > 0: the last step of a cycle; the back substitution over bk columns
// follows in the same thread (each rhs's state belongs to one thread)
__global__ void __launch_bounds__(256) k_gm_rotate(int nrhs, int j, const double* __restrict__ nrm2_in,
                                                    const double* __restrict__ part, int nb,
                                                    double* __restrict__ st, double* __restrict__ scale, int bk,
                                                    double* __restrict__ coef) {
  __shared__ double vals[FUSE_VALS];
  const double* __restrict__ nrm2 = small_reduction(nrhs * 2, 2, nrm2_in, part, nb, vals);
  int s = threadIdx.x;
  if (s >= nrhs) return;
  gm_rotate_rhs(s, j, nrm2, st, scale);
  if (bk > 0) gm_backsolve_rhs(s, bk, st, coef);
}

// The restart start (rotation < 0) or rotation j of the device GMRES fused
// with the scaled copy y = x / ||x|| that follows it: every block finishes
// the small reduction of the norms (same routine and order as the
// single-block kernels, so the same values), scales its part of x, and
// block (0, 0) also updates the state.  No block reads what another writes.
template <typename T>
__global__ void __launch_bounds__(256) k_gm_step_copy(int nrhs, int rotation, const double* __restrict__ part,
                                                       int nb, double* __restrict__ st, double* __restrict__ scale,
                                                       const cx<T>* __restrict__ x, cx<T>* __restrict__ y,
                                                       int64_t len) {
  __shared__ double vals[FUSE_VALS];
  const double* __restrict__ nrm2 = small_reduction(nrhs * 2, 2, nullptr, part, nb, vals);
  if (blockIdx.x == 0 && blockIdx.y == 0 && (int)threadIdx.x < nrhs) {
    if (rotation < 0) gm_start_rhs(threadIdx.x, nrm2, st, scale);
    else gm_rotate_rhs(threadIdx.x, rotation, nrm2, st, scale);
  }
  const int s = blockIdx.y;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= len) return;
  const double h = sqrt(nrm2[2 * s]);
  const double ar = h > 0 ? 1.0 / h : 0.0;
  const cx<T> xv = x[s * len + t];
  cx<T> out;
  out.re = (T)(ar * (double)xv.re);
  out.im = (T)(ar * (double)xv.im);
  y[s * len + t] = out;
}

int launch_gm_start(int nrhs, const double* nrm2, const double* part, int nb, double* st, double* scale,
                    hipStream_t s) {
  if (nrhs < 1 || nrhs > MAXRHS_KRYLOV || (part && nrhs * 2 > FUSE_VALS)) return (int)hipErrorInvalidValue;
  ELH_LAUNCH(k_gm_start, dim3(1), dim3(256), 0, s, nrhs, nrm2, part, nb, st, scale);
  return (int)hipGetLastError();
}
int launch_gm_hcol(int nrhs, int j, const double* dots, const double* part, int nb, double* st, double* coef,
                   hipStream_t s) {
  if (nrhs < 1 || nrhs > MAXRHS_KRYLOV || (part && nrhs * 2 * (j + 1) > FUSE_VALS)) return (int)hipErrorInvalidValue;
  ELH_LAUNCH(k_gm_hcol, dim3(1), dim3(256), 0, s, nrhs, j, dots, part, nb, st, coef);
  return (int)hipGetLastError();
}
int launch_gm_rotate(int nrhs, int j, const double* nrm2, const double* part, int nb, double* st, double* scale,
                     hipStream_t s, int bk, double* coef) {
  if (nrhs < 1 || nrhs > MAXRHS_KRYLOV || (part && nrhs * 2 > FUSE_VALS) || (bk > 0 && !coef))
    return (int)hipErrorInvalidValue;
  ELH_LAUNCH(k_gm_rotate, dim3(1), dim3(256), 0, s, nrhs, j, nrm2, part, nb, st, scale, bk, coef);
  return (int)hipGetLastError();
}
template <typename T>
int launch_gm_step_copy(int nrhs, int rotation, const double* part, int nb, double* st, double* scale, const void* x,
                        void* y, int64_t len, hipStream_t s) {
  if (nrhs < 1 || !part || nrhs * 2 > FUSE_VALS) return (int)hipErrorInvalidValue;
  ELH_LAUNCH((k_gm_step_copy<T>), dim3((unsigned)((len + 255) / 256), nrhs), dim3(256), 0, s, nrhs, rotation,
             part, nb, st, scale, (const cx<T>*)x, (cx<T>*)y, len);
  return (int)hipGetLastError();
}
template int launch_gm_step_copy<double>(int, int, const double*, int, double*, double*, const void*, void*, int64_t,
                                         hipStream_t);
template int launch_gm_step_copy<float>(int, int, const double*, int, double*, double*, const void*, void*, int64_t,
                                        hipStream_t);

// ---------------------------------------------------------------------------
// Receivers of the FWI misfit: the restriction P_r samples a wavefield at a
// list of storage indices (one unknown each), the injection P_r^T scatters
// receiver values back into a zero wavefield.  Indices outside the vector
// are skipped (sampled as zero).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_rec_sample(int64_t vs, int nrec, const int64_t* __restrict__ idx,
                                                     const cx<double>* __restrict__ u,
                                                     const cx<double>* __restrict__ dobs, cx<double>* __restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (i >= nrec) return;
  const int64_t j = idx[i];
  cx<double> v = (j >= 0 && j < vs) ? u[(int64_t)s * vs + j] : czero<double>();
  if (dobs) v = v - dobs[(int64_t)s * nrec + i];
  d[(int64_t)s * nrec + i] = v;
}

// phi[s] = 1/2 sum_i |r[s][i]|^2, one block per rhs, fixed-order tree
__global__ void __launch_bounds__(256) k_rec_half_norm2(int nrec, const cx<double>* __restrict__ r,
                                                         double* __restrict__ phi) {
  __shared__ double red[256];
  const int s = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < nrec; i += 256) acc += abs2(r[(int64_t)s * nrec + i]);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) phi[s] = 0.5 * red[0];
}

// phi[nrhs] = sum of phi[0..nrhs) in order (the total misfit)
__global__ void k_rec_total(int nrhs, double* __restrict__ phi) {
  if (threadIdx.x != 0) return;
  double t = 0.0;
  for (int s = 0; s < nrhs; ++s) t += phi[s];
  phi[nrhs] = t;
}

__global__ void __launch_bounds__(256) k_rec_inject(int64_t vs, int nrec, const int64_t* __restrict__ idx,
                                                     const cx<double>* __restrict__ r, double scale,
                                                     cx<double>* __restrict__ v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (i >= nrec) return;
  const int64_t j = idx[i];
  const cx<double> a = r[(int64_t)s * nrec + i];
  if (j >= 0 && j < vs) v[(int64_t)s * vs + j] = mk(scale * a.re, scale * a.im);
}

int launch_rec_sample(int64_t vs, int nrec, const int64_t* idx, const void* u, const void* dobs, void* d, double* phi,
                      int nrhs, hipStream_t st) {
  if (nrec < 1 || nrhs < 1 || nrhs > 65535) return (int)hipErrorInvalidValue;
  ELH_LAUNCH(k_rec_sample, dim3((nrec + 255) / 256, nrhs), dim3(256), 0, st, vs, nrec, idx, (const cx<double>*)u,
             (const cx<double>*)dobs, (cx<double>*)d);
  if (phi) {
    ELH_LAUNCH(k_rec_half_norm2, dim3(nrhs), dim3(256), 0, st, nrec, (const cx<double>*)d, phi);
    ELH_LAUNCH(k_rec_total, dim3(1), dim3(64), 0, st, nrhs, phi);
  }
  return (int)hipGetLastError();
}

int launch_rec_inject(int64_t vs, int nrec, const int64_t* idx, const void* r, double scale, void* v, int nrhs,
                      hipStream_t st) {
  if (nrec < 1 || nrhs < 1 || nrhs > 65535) return (int)hipErrorInvalidValue;
  ELH_LAUNCH(k_rec_inject, dim3((nrec + 255) / 256, nrhs), dim3(256), 0, st, vs, nrec, idx, (const cx<double>*)r,
             scale, (cx<double>*)v);
  return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Outer flexible GMRES with its bookkeeping on the device, one thread per
// right-hand side.  The basis stays unnormalised as in the host driver:
// V_i = v_i / sig_i, h_ij = sig_i sig_j <V_i, A Z_j>, h_{j+1,j} = sig_j
// ||V_{j+1}||, x += sum_j (y_j sig_j) Z_j.  Per rhs: the GM_STRIDE block
// (H, g, sines, cosines) followed by sig_0..sig_MAXDOT and the scalars
// below (GO_STRIDE doubles).  stat (4 doubles per rhs, copied to the host
// after every step): live, jend, residual estimate |g_{j+1}| / ||b||, bad.
// ---------------------------------------------------------------------------
constexpr int GO_SIG = GM_STRIDE, GO_NB = GO_SIG + MAXDOT + 1, GO_RTOL = GO_NB + 1, GO_LIVE = GO_NB + 2,
              GO_JEND = GO_NB + 3;
static_assert(GO_JEND < GO_STRIDE, "outer GMRES record");

__device__ inline double* go_rec(double* st, int s) { return st + (size_t)s * GO_STRIDE; }

// restart: g = (beta, 0, ...), sig_0 = 1/beta; par[4s..]: active, ||b||, rtol
__global__ void __launch_bounds__(256) k_go_start(int nrhs, const double* __restrict__ nrm2_in,
                                                   const double* __restrict__ part, int nb,
                                                   const double* __restrict__ par, double* __restrict__ st,
                                                   double* __restrict__ stat) {
  __shared__ double vals[FUSE_VALS];
  const double* __restrict__ nrm2 = small_reduction(nrhs * 2, 2, nrm2_in, part, nb, vals);
  const int s = threadIdx.x;
  if (s >= nrhs) return;
  double* r = go_rec(st, s);
  const double beta = sqrt(nrm2[2 * s]);
  const bool act = par[4 * s] != 0.0 && beta > 0;
  zc* g = gm_g(r, 0);
  for (int i = 0; i < MAXDOT; ++i) g[i] = {0.0, 0.0};
  g[0] = {beta, 0.0};
  r[GO_SIG] = act ? 1.0 / beta : 0.0;
  r[GO_NB] = par[4 * s + 1];
  r[GO_RTOL] = par[4 * s + 2];
  r[GO_LIVE] = act ? 1.0 : 0.0;
  r[GO_JEND] = -1.0;
  stat[4 * s] = r[GO_LIVE];
  stat[4 * s + 1] = -1.0;
  stat[4 * s + 2] = r[GO_NB] > 0 ? beta / r[GO_NB] : 0.0;
  stat[4 * s + 3] = isfinite(beta) ? 0.0 : 1.0;
}

// after the dots d_i = <V_i, A Z_j>: column j of H (live rhs) and the
// Gram-Schmidt coefficients -sig_i^2 d_i (every rhs)
__global__ void __launch_bounds__(256) k_go_hcol(int nrhs, int j, const double* __restrict__ dots_in,
                                                  const double* __restrict__ part, int nb, double* __restrict__ st,
                                                  double* __restrict__ coef) {
  __shared__ double vals[FUSE_VALS];
  const double* __restrict__ dots = small_reduction(nrhs * 2 * (j + 1), 2 * (j + 1), dots_in, part, nb, vals);
  const int s = threadIdx.x;
  if (s >= nrhs) return;
  double* r = go_rec(st, s);
  const bool live = r[GO_LIVE] != 0.0;
  const double sj = r[GO_SIG + j];
  for (int i = 0; i <= j; ++i) {
    const double dr = dots[(s * (j + 1) + i) * 2], di = dots[(s * (j + 1) + i) * 2 + 1];
    const double si = r[GO_SIG + i];
    if (live) *gm_H(r, 0, i, j) = {(si * sj) * dr, (si * sj) * di};
    coef[(s * (j + 1) + i) * 2] = -(si * si) * dr;
    coef[(s * (j + 1) + i) * 2 + 1] = -(si * si) * di;
  }
}

// after ||V_{j+1}||^2: sig_{j+1}; for live rhs the subdiagonal, the previous
// rotations, the new rotation, g, the residual estimate and the stop test
__global__ void __launch_bounds__(256) k_go_rotate(int nrhs, int j, const double* __restrict__ nrm2_in,
                                                    const double* __restrict__ part, int nb, double* __restrict__ st,
                                                    double* __restrict__ stat) {
  __shared__ double vals[FUSE_VALS];
  const double* __restrict__ nrm2 = small_reduction(nrhs * 2, 2, nrm2_in, part, nb, vals);
  const int s = threadIdx.x;
  if (s >= nrhs) return;
  double* r = go_rec(st, s);
  const double wn = sqrt(nrm2[2 * s]);
  const double sj = r[GO_SIG + j];
  r[GO_SIG + j + 1] = wn > 0 ? 1.0 / wn : 0.0;
  if (r[GO_LIVE] == 0.0) {
    stat[4 * s] = 0.0;
    return;
  }
  const double hn = sj * wn;
  if (!isfinite(hn)) {
    r[GO_LIVE] = 0.0;
    stat[4 * s] = 0.0;
    stat[4 * s + 3] = 1.0;
    return;
  }
  *gm_H(r, 0, j + 1, j) = {hn, 0.0};
  zc* sn = gm_sn(r, 0);
  double* cs = gm_cs(r, 0);
  for (int i = 0; i < j; ++i) {
    zc a = *gm_H(r, 0, i, j), b = *gm_H(r, 0, i + 1, j);
    zc t = zmul(sn[i], b);
    zc na = {cs[i] * a.re + t.re, cs[i] * a.im + t.im};
    zc u = zmul(zconj(sn[i]), a);
    zc nbv = {-u.re + cs[i] * b.re, -u.im + cs[i] * b.im};
    *gm_H(r, 0, i, j) = na;
    *gm_H(r, 0, i + 1, j) = nbv;
  }
  zc a = *gm_H(r, 0, j, j), b = *gm_H(r, 0, j + 1, j);
  double c;
  zc sg;
  const double aa = zabs(a), bb = zabs(b);
  if (bb == 0) { c = 1; sg = {0, 0}; }
  else if (aa == 0) { c = 0; sg = {b.re / bb, -b.im / bb}; }
  else {
    const double den = hypot(aa, bb);
    c = aa / den;
    const zc ph = {a.re / aa, a.im / aa};
    sg = zmul(ph, zc{b.re / den, -b.im / den});
  }
  cs[j] = c;
  sn[j] = sg;
  const zc t = zmul(sg, b);
  *gm_H(r, 0, j, j) = {c * a.re + t.re, c * a.im + t.im};
  *gm_H(r, 0, j + 1, j) = {0, 0};
  zc* g = gm_g(r, 0);
  const zc gj = g[j];
  const zc u = zmul(zconj(sg), gj);
  g[j + 1] = {-u.re, -u.im};
  g[j] = {c * gj.re, c * gj.im};
  r[GO_JEND] = j;
  const double res = zabs(g[j + 1]) / r[GO_NB];
  const bool stop = res <= r[GO_RTOL] || hn == 0;
  if (stop) r[GO_LIVE] = 0.0;
  stat[4 * s] = stop ? 0.0 : 1.0;
  stat[4 * s + 1] = j;
  stat[4 * s + 2] = res;
  stat[4 * s + 3] = 0.0;
}

// end of a restart: y = R^{-1} g over the jend+1 columns of each rhs, and
// the update coefficients y_i sig_i (zero beyond jend, all zero for a rhs
// that took no step), k per rhs in coef
__global__ void k_go_update(int nrhs, int k, const double* __restrict__ st, double* __restrict__ coef) {
  const int s = threadIdx.x;
  if (s >= nrhs) return;
  double* r = const_cast<double*>(st) + (size_t)s * GO_STRIDE;
  const int kk = (int)r[GO_JEND] + 1;
  const zc* g = gm_g(r, 0);
  zc y[MAXDOT];
  for (int i = kk - 1; i >= 0; --i) {
    zc acc = g[i];
    for (int q = i + 1; q < kk; ++q) {
      const zc t = zmul(*gm_H(r, 0, i, q), y[q]);
      acc.re -= t.re;
      acc.im -= t.im;
    }
    const zc d = *gm_H(r, 0, i, i);
    const double dd = d.re * d.re + d.im * d.im;
    y[i] = dd > 0 ? zc{(acc.re * d.re + acc.im * d.im) / dd, (acc.im * d.re - acc.re * d.im) / dd} : zc{0, 0};
  }
  for (int i = 0; i < k; ++i) {
    const double sg = i < kk ? r[GO_SIG + i] : 0.0;
    coef[(s * k + i) * 2] = i < kk ? y[i].re * sg : 0.0;
    coef[(s * k + i) * 2 + 1] = i < kk ? y[i].im * sg : 0.0;
  }
}

int launch_go_start(int nrhs, const double* nrm2, const double* part, int nb, const double* par, double* st,
                    double* stat, hipStream_t s) {
  if (nrhs < 1 || nrhs > MAXRHS_KRYLOV || (part && nrhs * 2 > FUSE_VALS)) return (int)hipErrorInvalidValue;
  ELH_LAUNCH(k_go_start, dim3(1), dim3(256), 0, s, nrhs, nrm2, part, nb, par, st, stat);
  return (int)hipGetLastError();
}
int launch_go_hcol(int nrhs, int j, const double* dots, const double* part, int nb, double* st, double* coef,
                   hipStream_t s) {
  if (nrhs < 1 || nrhs > MAXRHS_KRYLOV || j + 1 >= MAXDOT || (part && nrhs * 2 * (j + 1) > FUSE_VALS))
    return (int)hipErrorInvalidValue;
  ELH_LAUNCH(k_go_hcol, dim3(1), dim3(256), 0, s, nrhs, j, dots, part, nb, st, coef);
  return (int)hipGetLastError();
}
int launch_go_rotate(int nrhs, int j, const double* nrm2, const double* part, int nb, double* st, double* stat,
                     hipStream_t s) {
  if (nrhs < 1 || nrhs > MAXRHS_KRYLOV || j + 1 >= MAXDOT || (part && nrhs * 2 > FUSE_VALS))
    return (int)hipErrorInvalidValue;
  ELH_LAUNCH(k_go_rotate, dim3(1), dim3(256), 0, s, nrhs, j, nrm2, part, nb, st, stat);
  return (int)hipGetLastError();
}
int launch_go_update(int nrhs, int k, const double* st, double* coef, hipStream_t s) {
  if (nrhs < 1 || nrhs > MAXRHS_KRYLOV || k < 1 || k >= MAXDOT) return (int)hipErrorInvalidValue;
  ELH_LAUNCH(k_go_update, dim3(1), dim3(64), 0, s, nrhs, k, st, coef);
  return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Dense coarsest-level solve (the paper's LU choice for 2D): the shifted
// operator is assembled by applying it to unit vectors, inverted once by
// Gauss-Jordan elimination with partial pivoting, and applied as a dense
// matrix-vector product.  A is row-major N x N (A = H^T after assembly).
// ---------------------------------------------------------------------------
__global__ void k_unit_vectors(int64_t N, cx<double>* __restrict__ E) {
  // E: N vectors of length N, E[j][i] = (i == j)
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * N) return;
  int64_t j = t / N, i = t % N;
  E[t] = mk(i == j ? 1.0 : 0.0, 0.0);
}

// rows of A (= columns of H) that are boundary faces: identity
__global__ void k_fix_boundary_rows(int64_t N, const int* __restrict__ isb, cx<double>* __restrict__ A) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  if (isb[i]) A[i * N + i] = mk(1.0, 0.0);
}

__global__ void k_gj_pivot(int64_t N, int64_t k, const cx<double>* __restrict__ A, int* __restrict__ piv,
                           cx<double>* __restrict__ pval) {
  __shared__ double best[256];
  __shared__ int64_t arg[256];
  double b = -1.0;
  int64_t a = k;
  for (int64_t i = k + threadIdx.x; i < N; i += blockDim.x) {
    double v = abs2(A[i * N + k]);
    if (v > b) { b = v; a = i; }
  }
  best[threadIdx.x] = b;
  arg[threadIdx.x] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      double ob = best[threadIdx.x + o];
      int64_t oa = arg[threadIdx.x + o];
      if (ob > best[threadIdx.x] || (ob == best[threadIdx.x] && oa < arg[threadIdx.x])) {
        best[threadIdx.x] = ob;
        arg[threadIdx.x] = oa;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    piv[0] = (int)arg[0];
    pval[0] = A[arg[0] * N + k];  // read before any block of the swap kernel writes
  }
}

// swap rows k and piv of [A | B], scale row k by 1/pivot, save column k
__global__ void k_gj_swap_scale(int64_t N, int64_t k, const int* __restrict__ piv, cx<double>* __restrict__ A,
                                cx<double>* __restrict__ B, const cx<double>* __restrict__ pval) {
  const int64_t p = piv[0];
  const cx<double> pv = pval[0];
  const double ip = 1.0 / abs2(pv);
  const cx<double> r = mk(pv.re * ip, -pv.im * ip);
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < 2 * N; j += (int64_t)gridDim.x * blockDim.x) {
    cx<double>* M = j < N ? A : B;
    const int64_t jj = j < N ? j : j - N;
    cx<double> vk = M[k * N + jj], vp = M[p * N + jj];
    if (p != k) M[p * N + jj] = vk;
    M[k * N + jj] = vp * r;
  }
}

__global__ void k_gj_column(int64_t N, int64_t k, const cx<double>* __restrict__ A, cx<double>* __restrict__ col) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) col[i] = (i == k) ? czero<double>() : A[i * N + k];
}

__global__ void k_gj_eliminate(int64_t N, int64_t k, const cx<double>* __restrict__ col, cx<double>* __restrict__ A,
                               cx<double>* __restrict__ B) {
  const int64_t i = blockIdx.y;
  const cx<double> f = col[i];
  if (f.re == 0.0 && f.im == 0.0) return;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < 2 * N; j += (int64_t)gridDim.x * blockDim.x) {
    if (j < N) {
      if (j >= k) A[i * N + j] -= f * A[k * N + j];
    } else {
      B[i * N + (j - N)] -= f * B[k * N + (j - N)];
    }
  }
}

int launch_dense_assemble_prep(int64_t N, void* E, hipStream_t st) {
  ELH_LAUNCH(k_unit_vectors, dim3((unsigned)((N * N + 255) / 256)), dim3(256), 0, st, N, (cx<double>*)E);
  return (int)hipGetLastError();
}
int launch_dense_fix(int64_t N, const int* isb, void* A, hipStream_t st) {
  ELH_LAUNCH(k_fix_boundary_rows, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, N, isb,
                     (cx<double>*)A);
  return (int)hipGetLastError();
}
// Gauss-Jordan inverse: A is destroyed, B (identity on entry) becomes A^{-1}
int launch_dense_invert(int64_t N, void* A, void* B, void* col, int* piv, hipStream_t st) {
  cx<double>* a = (cx<double>*)A;
  cx<double>* b = (cx<double>*)B;
  cx<double>* c = (cx<double>*)col;
  ELH_LAUNCH(k_unit_vectors, dim3((unsigned)((N * N + 255) / 256)), dim3(256), 0, st, N, b);
  for (int64_t k = 0; k < N; ++k) {
    // col has N+1 entries: col[N] carries the pivot value
    ELH_LAUNCH(k_gj_pivot, dim3(1), dim3(256), 0, st, N, k, (const cx<double>*)a, piv, c + N);
    ELH_LAUNCH(k_gj_swap_scale, dim3((unsigned)((2 * N + 255) / 256)), dim3(256), 0, st, N, k,
                       (const int*)piv, a, b, (const cx<double>*)(c + N));
    ELH_LAUNCH(k_gj_column, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, N, k,
                       (const cx<double>*)a, c);
    unsigned gx = (unsigned)((2 * N + 255) / 256);
    if (gx > 16) gx = 16;
    ELH_LAUNCH(k_gj_eliminate, dim3(gx, (unsigned)N), dim3(256), 0, st, N, k, (const cx<double>*)c, a, b);
  }
  return (int)hipGetLastError();
}

// x[s] = op(Q) b[s] with Q row-major N x N.  transposed: x_i = sum_j Q[j][i] b_j
// (coalesced over i); otherwise x_i = sum_j conj?(Q[i][j]) b_j.
template <typename T>
__global__ void __launch_bounds__(256) k_dense_mv(int64_t N, const cx<T>* __restrict__ Q, int transposed, int cj,
                                                   const cx<T>* __restrict__ b, cx<T>* __restrict__ x, int nrhs) {
  const int s = blockIdx.y;
  const cx<T>* bs = b + (int64_t)s * N;
  if (transposed) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    cx<T> acc = czero<T>();
    for (int64_t j = 0; j < N; ++j) {
      cx<T> q = Q[j * N + i];
      if (cj) q = conj(q);
      acc += q * bs[j];
    }
    x[(int64_t)s * N + i] = acc;
  } else {
    // one wavefront per row
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    if (row >= N) return;
    cx<T> acc = czero<T>();
    for (int64_t j = lane; j < N; j += 64) {
      cx<T> q = Q[row * N + j];
      if (cj) q = conj(q);
      acc += q * bs[j];
    }
    for (int o = 32; o > 0; o >>= 1) {
      acc.re += __shfl_down(acc.re, o);
      acc.im += __shfl_down(acc.im, o);
    }
    if (lane == 0) x[(int64_t)s * N + row] = acc;
  }
}

template <typename T>
int launch_dense_mv(int64_t N, const void* Q, int transposed, int cj, const void* b, void* x, int nrhs,
                    hipStream_t st) {
  if (transposed)
    ELH_LAUNCH((k_dense_mv<T>), dim3((unsigned)((N + 255) / 256), nrhs), dim3(256), 0, st, N,
                       (const cx<T>*)Q, 1, cj, (const cx<T>*)b, (cx<T>*)x, nrhs);
  else
    ELH_LAUNCH((k_dense_mv<T>), dim3((unsigned)((N + 3) / 4), nrhs), dim3(256), 0, st, N, (const cx<T>*)Q,
                       0, cj, (const cx<T>*)b, (cx<T>*)x, nrhs);
  return (int)hipGetLastError();
}
template int launch_dense_mv<double>(int64_t, const void*, int, int, const void*, void*, int, hipStream_t);
template int launch_dense_mv<float>(int64_t, const void*, int, int, const void*, void*, int, hipStream_t);

__global__ void k_fill_zero(uint2* p, int64_t n8) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n8; i += (int64_t)gridDim.x * blockDim.x) p[i] = make_uint2(0, 0);
}
int launch_zero(void* p, int64_t bytes, hipStream_t st) {
  // every vector here is a whole number of 8-byte complex64 entries or wider
  int64_t n8 = bytes / 8;
  if (n8 == 0) return 0;
  int64_t nb = (n8 + 255) / 256;
  if (nb > 65536) nb = 65536;
  ELH_LAUNCH(k_fill_zero, dim3((unsigned)nb), dim3(256), 0, st, (uint2*)p, n8);
  return (int)hipGetLastError();
}

}  // namespace elh
