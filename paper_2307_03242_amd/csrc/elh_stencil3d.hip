// Tuned 3D apply / residual of H^beta (forward operator, any level) for
// gfx950.
//
// Arithmetic (Section 3.1, eq. mixed-discretized; Section 5.3 eqs.
// dxSkew3D, massHO3D): the beta-spread derivative of u_k along x_l is
// D_l S_l u_k with the spread S_l = beta*I + (1-beta) * prod_{a != l} A_a
// (A_a = (1/4)[1 2 1] along x_a, zero outside).  S_l acts on the axes
// other than l, so it commutes with the difference D_l: we form the
// "spread fields" Y_kl = S_l u_k once per point and take plain two-point
// differences of them.  The flux through a face is mu_e * (Y(hi) - Y(lo))/h
// and the output row is the difference of the two fluxes beside it.
//
// Data flow (2.5D blocking): a workgroup of 64 x 6 threads owns a 64 x 6
// column window of the x_1-x_2 plane and marches along x_3.  Lanes 0 and
// 63 and rows 0 and 5 are halo columns: they load and derive data but
// write no output, so the workgroup produces 62 x 4 outputs per plane.
// Along x_3 every column keeps rolling register windows (u_k at three
// planes, Y_k3, rho-weighted u_k for the spread mass, averaged mu);
// neighbours in the plane come from LDS; each of the three barrier-separated
// phases of a plane handles all displacement components.  Tiles are numbered so that the
// workgroups of one XCD (blockIdx mod 8) sweep a contiguous block of tiles
// and share halo columns in their L2.
#include "elh_device.h"
#include "elh_internal.h"

namespace elh {

constexpr int ST_TX = 64;             // slots along x_1 (one wavefront)
constexpr int ST_OX = ST_TX - 2;      // outputs along x_1

template <typename T, int ST_TY> struct Tile3 {
  cx<T> R[3][ST_TY][ST_TX];    // raw u_k(t+1)
  cx<T> Z[3][ST_TY][ST_TX];    // A_3 u_k(t)
  cx<T> B1[3][ST_TY][ST_TX];   // A_1 u_k(t+1)
  cx<T> Y1[3][ST_TY][ST_TX];   // Y_k1(t)
  cx<T> Y2[3][ST_TY][ST_TX];   // Y_k2(t)
  cx<T> W[3][ST_TY][ST_TX];    // rho_f u_k (t)
  cx<T> P[ST_TY][ST_TX];    // p(t)
  T Mn[ST_TY][ST_TX];       // mu(t+1)
  T Rn[ST_TY][ST_TX];       // rho(t+1)
  T M[ST_TY][ST_TX];        // mu(t)
  T MX[ST_TY][ST_TX];       // mean of mu over x_1 pairs (t)
  T MY[ST_TY][ST_TX];       // mean of mu over x_2 pairs (t)
  T MZ[ST_TY][ST_TX];       // mean of mu over x_3 pairs (t)
};

// Workgroup barrier for LDS hand-off only: wait for this wave's LDS
// operations (lgkmcnt = 0, vmcnt and expcnt left at their maxima) and meet
// at s_barrier.  Unlike __syncthreads() it does not drain the global loads
// that prefetch the next x_3 plane, so they stay in flight across phases.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_s_barrier();
}

template <typename T>
__device__ __forceinline__ cx<T> ldu(const cx<T>* __restrict__ f, int64_t fs, int64_t idx, bool ok) {
  return ok ? f[idx] : czero<T>();
}

// One axis of the absorbing-layer profile: amp * (delta/width)^2 with delta
// the distance into the layer at physical coordinate xp along an axis of
// physical length len (zero in the interior).
template <typename T>
__device__ __forceinline__ T absorb_axis(T xp, T len, T w, T iw, T amp) {
  T d = (w - xp > T(0) ? w - xp : T(0)) + (xp - (len - w) > T(0) ? xp - (len - w) : T(0));
  T r = d * iw;
  return amp * r * r;
}

template <typename T, bool RESID, int ST_TY>
__global__ void __launch_bounds__(ST_TX * ST_TY)
k_apply3d_tiled(LevelArgs<T> L, const cx<T>* __restrict__ x, const cx<T>* __restrict__ b, cx<T>* __restrict__ y,
                int tiles_x, int tiles_y, int nzc, int zc, int ntiles, int per_xcd) {
  constexpr int ST_OY = ST_TY - 2;      // outputs along x_2
  __shared__ Tile3<T, ST_TY> S;
  // XCD-aware tile number: workgroups are dealt round-robin to the 8 XCDs
  const int bid = blockIdx.x;
  const int tile = (bid & 7) * per_xcd + (bid >> 3);
  if (tile >= ntiles) return;
  int rest = tile;
  const int tx = rest % tiles_x; rest /= tiles_x;
  const int ty = rest % tiles_y; rest /= tiles_y;
  const int tz = rest % nzc; rest /= nzc;
  const int s = rest;                              // right-hand side
  const int lane = threadIdx.x, row = threadIdx.y;
  const int n1 = L.n[0], n2 = L.n[1], n3 = L.n[2];
  const int c1 = tx * ST_OX - 1 + lane;
  const int c2 = ty * ST_OY - 1 + row;
  const int z0 = tz * zc;
  const int z1 = min(z0 + zc, n3);
  const bool inplane = c1 >= 0 && c1 < n1 && c2 >= 0 && c2 < n2;
  const bool inner_row = row >= 1 && row <= ST_OY;   // whole wavefronts: uniform branches
  const bool outslot = lane >= 1 && lane <= ST_OX && inner_row && inplane;
  const int cc1 = min(max(c1, 0), n1 - 1), cc2 = min(max(c2, 0), n2 - 1);  // clamped (media)
  const int64_t fs = L.fs;
  const int64_t plane = (int64_t)n1 * n2;
  const int64_t col = (int64_t)cc2 * n1 + cc1;
  const cx<T>* xs = x + (int64_t)s * L.vs;
  const cx<T>* bs = RESID ? b + (int64_t)s * L.vs : nullptr;
  cx<T>* ys = y + (int64_t)s * L.vs;
  const int lm = lane > 0 ? lane - 1 : 0, lp = lane < ST_TX - 1 ? lane + 1 : ST_TX - 1;
  const int rm = row > 0 ? row - 1 : 0, rp = row < ST_TY - 1 ? row + 1 : ST_TY - 1;
  const T beta = L.beta, omb = T(1) - L.beta, q = T(0.25);
  const T ih = L.ih, ih2 = L.ih * L.ih;
  const T cn = omb / T(6);
  // absorbing layer: gamma~ at a face = gamma (+alpha) + sum over axes of a
  // one-axis profile; the x_1 and x_2 parts are fixed along the x_3 march
  const bool has_abl = L.abl_w > T(0) && L.abl_amp != T(0);
  const T abl_iw = L.abl_iw;
  const T len1 = n1 * L.h, len2 = n2 * L.h, len3 = n3 * L.h;
  T g1f = L.gam, g2f = L.gam, g3f = L.gam;  // constant parts for u_1, u_2, u_3 faces
  if (has_abl) {
    const T a1c = absorb_axis<T>((T(c1) + T(0.5)) * L.h, len1, L.abl_w, abl_iw, L.abl_amp);
    const T a1f = absorb_axis<T>(T(c1) * L.h, len1, L.abl_w, abl_iw, L.abl_amp);
    const T a2c = absorb_axis<T>((T(c2) + T(0.5)) * L.h, len2, L.abl_w, abl_iw, L.abl_amp);
    const T a2f = absorb_axis<T>(T(c2) * L.h, len2, L.abl_w, abl_iw, L.abl_amp);
    g1f += a1f + a2c;
    g2f += a1c + a2f;
    g3f += a1c + a2c;
  }
  // Loads always read a valid (clamped) address; whether the value is a
  // real unknown (inside the grid, not a boundary face) is a separate mask
  // applied when the value enters its register window.  A masked load would
  // be a branch + select that makes the wave wait for the prefetch at once.
  auto u_ok = [&](int k, int z) -> bool {
    bool ok = inplane && z >= 0 && z < n3;
    if (k == 0) ok = ok && c1 > 0;
    if (k == 1) ok = ok && c2 > 0;
    if (k == 2) ok = ok && z > 0;
    return ok;
  };
  auto load_raw = [&](int f, int z) -> cx<T> {
    int zz = min(max(z, 0), n3 - 1);
    return xs[f * fs + (int64_t)zz * plane + col];
  };
  auto load_u = [&](int k, int z) -> cx<T> { return u_ok(k, z) ? load_raw(k, z) : czero<T>(); };
  auto load_p = [&](int z) -> cx<T> { return (inplane && z >= 0 && z < n3) ? load_raw(3, z) : czero<T>(); };
  auto load_m = [&](const T* m, int z) -> T {
    int zz = min(max(z, 0), n3 - 1);
    return m[(int64_t)zz * plane + col];
  };
  // rho of the column beside the halo slot (lane 0: x_1 - 1; row 0: x_2 - 1):
  // the face average of rho there needs one column beyond the tile
  const int64_t side_col = lane == 0 ? (int64_t)cc2 * n1 + max(cc1 - 1, 0)
                                     : (int64_t)max(cc2 - 1, 0) * n1 + cc1;
  auto load_side_rho = [&](int z) -> T {
    int zz = min(max(z, 0), n3 - 1);
    return L.rho[(int64_t)zz * plane + side_col];
  };

  // register windows (see the loop invariant below)
  cx<T> U[3][3], Y3[3][3], W[3][3];
  T MU[3], RHO[2], MX[3], MY[3];
  cx<T> P0, PM;
  T KAP;
  const int t0 = z0 - 2;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    U[k][0] = czero<T>();
    U[k][1] = czero<T>();
    U[k][2] = load_u(k, t0 + 1);
    Y3[k][0] = Y3[k][1] = Y3[k][2] = czero<T>();
    W[k][0] = W[k][1] = W[k][2] = czero<T>();
  }
  MU[0] = MU[1] = load_m(L.mu, t0);
  MU[2] = load_m(L.mu, t0 + 1);
  RHO[0] = load_m(L.rho, t0);
  RHO[1] = load_m(L.rho, t0 + 1);
  T RHOS = load_side_rho(t0 + 1);
  MX[0] = MX[1] = MX[2] = MU[0];
  MY[0] = MY[1] = MY[2] = MU[0];
  P0 = load_p(t0);
  PM = czero<T>();
  KAP = load_m(L.kap, t0);

#pragma unroll 3
  for (int t = t0; t < z1; ++t) {
    // loop invariant: U[k] = u_k(t-1..t+1), Y3/W/MX/MY valid at t-1, t;
    // MU = mu(t-1..t+1), RHO = rho(t), rho(t+1), P0 = p(t), PM = p(t-1)
    // prefetch plane t+2 (and p, kappa at t+1)
    cx<T> un[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) un[k] = load_raw(k, t + 2);
    const T mun = load_m(L.mu, t + 2);
    const T rhon = load_m(L.rho, t + 2);
    const T rhosn = load_side_rho(t + 2);
    const cx<T> pn = load_raw(3, t + 1);
    const T kapn = load_m(L.kap, t + 1);
    const bool emit = outslot && t >= z0;
    // right-hand side of plane t for the residual, fetched with the plane
    // prefetch so it is in flight during the phases below
    cx<T> bq[4];
    if (RESID) {
      const int64_t o = (int64_t)min(max(t, 0), n3 - 1) * plane + col;
#pragma unroll
      for (int f = 0; f < 4; ++f) bq[f] = bs[f * fs + o];
    }
    T a3c = T(0), a3f = T(0);
    if (has_abl) {
      a3c = absorb_axis<T>((T(t) + T(0.5)) * L.h, len3, L.abl_w, abl_iw, L.abl_amp);
      a3f = absorb_axis<T>(T(t) * L.h, len3, L.abl_w, abl_iw, L.abl_amp);
    }

    // phase A: media, pressure, raw u_k(t+1), A_3 u_k(t), rho-weighted u_k(t)
    S.Mn[row][lane] = MU[2];
    S.Rn[row][lane] = RHO[1];
    S.P[row][lane] = P0;
    S.M[row][lane] = MU[1];
    S.MX[row][lane] = MX[1];
    S.MY[row][lane] = MY[1];
    const T MZ = T(0.5) * (MU[0] + MU[1]);
    S.MZ[row][lane] = MZ;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      S.R[k][row][lane] = U[k][2];
      S.Z[k][row][lane] = q * (U[k][0] + U[k][2]) + T(0.5) * U[k][1];
      S.W[k][row][lane] = W[k][1];
    }
    lds_barrier();
    // phase B: face-averaged media and rho-weighted u_k at t+1; A_1 u(t+1),
    // Y_k1(t) = S_1 u(t), Y_k2(t) = S_2 u(t)
    MX[2] = T(0.5) * (S.Mn[row][lm] + MU[2]);
    MY[2] = T(0.5) * (S.Mn[rm][lane] + MU[2]);
    {
      const T rf1 = T(0.5) * ((lane == 0 ? RHOS : S.Rn[row][lm]) + RHO[1]);
      const T rf2 = T(0.5) * ((row == 0 ? RHOS : S.Rn[rm][lane]) + RHO[1]);
      const T rf3 = T(0.5) * (RHO[0] + RHO[1]);
      W[0][2] = rf1 * U[0][2];
      W[1][2] = rf2 * U[1][2];
      W[2][2] = rf3 * U[2][2];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const cx<T> Zk = S.Z[k][row][lane];
      S.B1[k][row][lane] = q * (S.R[k][row][lm] + S.R[k][row][lp]) + T(0.5) * U[k][2];
      if (inner_row)  // Y_k1 is only read along x_1, by the output rows
        S.Y1[k][row][lane] = beta * U[k][1] + omb * (q * (S.Z[k][rm][lane] + S.Z[k][rp][lane]) + T(0.5) * Zk);
      S.Y2[k][row][lane] = beta * U[k][1] + omb * (q * (S.Z[k][row][lm] + S.Z[k][row][lp]) + T(0.5) * Zk);
    }
    lds_barrier();
    // phase C: Y_k3(t+1) = S_3 u(t+1), then the rows of plane t
    cx<T> div = czero<T>();
    cx<T> out[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (inner_row) {  // Y_k3 only feeds the own column's output
        const cx<T> b1 = S.B1[k][row][lane];
        Y3[k][2] = beta * U[k][2] + omb * (q * (S.B1[k][rm][lane] + S.B1[k][rp][lane]) + T(0.5) * b1);
      }
      if (emit) {
        const cx<T> y1 = S.Y1[k][row][lane], y2 = S.Y2[k][row][lane];
        const cx<T> y1m = S.Y1[k][row][lm], y1p = S.Y1[k][row][lp];
        const cx<T> y2m = S.Y2[k][rm][lane], y2p = S.Y2[k][rp][lane];
        cx<T> acc;
        T g;  // gamma~ at the output face
        if (k == 0) {
          // d/dx1 (cell fluxes), d/dx2 and d/dx3 (edge fluxes, mu averaged over x1 pairs)
          acc = ih2 * (S.M[row][lm] * (y1 - y1m) - MU[1] * (y1p - y1));
          const T mlo = T(0.5) * (S.MX[rm][lane] + MX[1]), mhi = T(0.5) * (MX[1] + S.MX[rp][lane]);
          acc += ih2 * (mlo * (y2 - y2m) - mhi * (y2p - y2));
          const T zlo = T(0.5) * (MX[0] + MX[1]), zhi = T(0.5) * (MX[1] + MX[2]);
          acc += ih2 * (zlo * (Y3[0][1] - Y3[0][0]) - zhi * (Y3[0][2] - Y3[0][1]));
          acc += ih * (P0 - S.P[row][lm]);
          div += ih * (y1p - y1);
          g = g1f + a3c;
        } else if (k == 1) {
          acc = ih2 * (S.M[rm][lane] * (y2 - y2m) - MU[1] * (y2p - y2));
          const T mlo = T(0.5) * (S.MY[row][lm] + MY[1]), mhi = T(0.5) * (MY[1] + S.MY[row][lp]);
          acc += ih2 * (mlo * (y1 - y1m) - mhi * (y1p - y1));
          const T zlo = T(0.5) * (MY[0] + MY[1]), zhi = T(0.5) * (MY[1] + MY[2]);
          acc += ih2 * (zlo * (Y3[1][1] - Y3[1][0]) - zhi * (Y3[1][2] - Y3[1][1]));
          acc += ih * (P0 - S.P[rm][lane]);
          div += ih * (y2p - y2);
          g = g2f + a3c;
        } else {
          acc = ih2 * (MU[0] * (Y3[2][1] - Y3[2][0]) - MU[1] * (Y3[2][2] - Y3[2][1]));
          const T xlo = T(0.5) * (S.MZ[row][lm] + MZ), xhi = T(0.5) * (MZ + S.MZ[row][lp]);
          acc += ih2 * (xlo * (y1 - y1m) - xhi * (y1p - y1));
          const T ylo = T(0.5) * (S.MZ[rm][lane] + MZ), yhi = T(0.5) * (MZ + S.MZ[rp][lane]);
          acc += ih2 * (ylo * (y2 - y2m) - yhi * (y2p - y2));
          acc += ih * (P0 - PM);
          div += ih * (Y3[2][2] - Y3[2][1]);
          g = g3f + a3f;
        }
        // spread mass with the attenuation of the output face
        const cx<T> nb = S.W[k][row][lm] + S.W[k][row][lp] + S.W[k][rm][lane] + S.W[k][rp][lane] +
                         W[k][0] + W[k][2];
        const cx<T> sm = beta * W[k][1] + cn * nb;
        const cx<T> mf = mk(L.omega2, -L.omega2 * g);
        acc -= mf * sm;
        out[k] = acc;
      }
    }
    lds_barrier();
    if (emit) {
      const int64_t o = (int64_t)t * plane + (int64_t)c2 * n1 + c1;
      const bool face[3] = {c1 > 0, c2 > 0, t > 0};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        cx<T> v = face[k] ? out[k] : czero<T>();
        if (RESID && face[k]) v = bq[k] - v;
        ys[k * fs + o] = v;
      }
      cx<T> vp = div + KAP * P0;
      if (RESID) vp = bq[3] - vp;
      ys[3 * fs + o] = vp;
    }
    // advance the windows
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      U[k][0] = U[k][1]; U[k][1] = U[k][2]; U[k][2] = u_ok(k, t + 2) ? un[k] : czero<T>();
      Y3[k][0] = Y3[k][1]; Y3[k][1] = Y3[k][2];
      W[k][0] = W[k][1]; W[k][1] = W[k][2];
    }
    MU[0] = MU[1]; MU[1] = MU[2]; MU[2] = mun;
    RHO[0] = RHO[1]; RHO[1] = rhon;
    RHOS = rhosn;
    MX[0] = MX[1]; MX[1] = MX[2];
    MY[0] = MY[1]; MY[1] = MY[2];
    PM = P0; P0 = (inplane && t + 1 < n3) ? pn : czero<T>();
    KAP = kapn;
  }
}

template <typename T, int TY>
static int launch_tiled_ty(const LevelArgs<T>& L, const void* x, const void* b, void* y, int nrhs, int zc,
                           hipStream_t st) {
  constexpr int OY = TY - 2;
  const int tiles_x = (L.n[0] + ST_OX - 1) / ST_OX;
  const int tiles_y = (L.n[1] + OY - 1) / OY;
  if (zc <= 0) zc = 32;
  // keep at least ~2048 workgroups in flight: shorter x_3 chunks on small grids
  {
    int64_t cols = (int64_t)tiles_x * tiles_y * nrhs;
    int64_t want = (int64_t)L.n[2] * cols / 2048;
    if (want < zc) zc = (int)(want < 4 ? 4 : want);
  }
  if (zc > L.n[2]) zc = L.n[2];
  const int nzc = (L.n[2] + zc - 1) / zc;
  const int64_t ntiles64 = (int64_t)tiles_x * tiles_y * nzc * nrhs;
  if (ntiles64 > (1ll << 30)) return (int)hipErrorInvalidValue;
  const int ntiles = (int)ntiles64;
  const int per_xcd = (ntiles + 7) / 8;
  dim3 blk(ST_TX, TY), grd(8 * per_xcd);
  if (b)
    hipLaunchKernelGGL((k_apply3d_tiled<T, true, TY>), grd, blk, 0, st, L, (const cx<T>*)x, (const cx<T>*)b,
                       (cx<T>*)y, tiles_x, tiles_y, nzc, zc, ntiles, per_xcd);
  else
    hipLaunchKernelGGL((k_apply3d_tiled<T, false, TY>), grd, blk, 0, st, L, (const cx<T>*)x,
                       (const cx<T>*)nullptr, (cx<T>*)y, tiles_x, tiles_y, nzc, zc, ntiles, per_xcd);
  return (int)hipGetLastError();
}

// ty: tile height in slots (6 or 10; float64 always uses 6 for its LDS size)
template <typename T>
int launch_apply3d_tiled(const LevelArgs<T>& L, const void* x, const void* b, void* y, int nrhs, int zc, int ty,
                         hipStream_t st) {
  if constexpr (sizeof(T) == 4) {
    if (ty == 10) return launch_tiled_ty<T, 10>(L, x, b, y, nrhs, zc, st);
  }
  return launch_tiled_ty<T, 6>(L, x, b, y, nrhs, zc, st);
}
template int launch_apply3d_tiled<double>(const LevelArgs<double>&, const void*, const void*, void*, int, int, int,
                                          hipStream_t);
template int launch_apply3d_tiled<float>(const LevelArgs<float>&, const void*, const void*, void*, int, int, int,
                                         hipStream_t);

}  // namespace elh
