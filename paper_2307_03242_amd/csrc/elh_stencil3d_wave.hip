// Barrier-light 3D apply / residual of H^beta (forward operator) for gfx950.
//
// Same arithmetic as the point-wise kernel (Section 3.1, eq.
// mixed-discretized; Section 5.3, eqs. dxSkew3D, massHO3D), organised for
// the CDNA4 execution model:
//  * a workgroup of three wavefronts owns one x_2 row of a 64-wide x_1
//    segment and marches along x_3; wavefront k computes the rows of
//    u_{k+1} (the u-u block of H is diagonal in the component) and its
//    term of the divergence in the p row; lanes 0 and 63 are halo lanes
//    (62 outputs per wavefront); a remainder of at most 14 cells at the end
//    of the rows goes to workgroups whose wavefronts split into four 16-lane
//    groups, one row each (at n_1 = 256: 4.25 wavefronts per row, not 5);
//  * neighbours along x_1 are other lanes of the same wavefront, read with
//    DPP wavefront shifts;
//  * neighbours along x_2 (rows c-1, c+1; rho also at c-2) are loaded
//    directly; the segments of four neighbouring rows run on the same XCD
//    (tile order below), so these loads hit its L2, while the eight XCDs
//    work through the same x_3 chunk at once;
//  * along x_3 each wavefront keeps rolling register windows of its one
//    component (u at rows c-1..c+1, planes t-1 and t; the spread field Y_3;
//    the carried x_3 flux; the rho-weighted u of the spread mass; mu; p);
//  * the three divergence terms meet in LDS once per plane (one barrier,
//    double-buffered by plane parity) and wavefront 0 writes the p row.
// With S_l = beta*I + (1-beta) prod_{a != l} A_a (A_a = (1/4)[1 2 1] along
// x_a) the fields Y_l = S_l u are formed once per point; the flux through a
// face is mu_e (Y(hi) - Y(lo)) / h and the row is the difference of the two
// fluxes beside it, as in the point-wise kernel.
#include "elh_device.h"
#include "elh_internal.h"

namespace elh {

namespace {

constexpr int WV_LANES = 64;
constexpr int WV_OUT = WV_LANES - 2;   // outputs per wave along x_1
// x_1 remainders of at most RG_OUT cells go to wavefronts of four 16-lane
// groups, one x_2 row each (14 outputs per group)
constexpr int RG_LANES = 16;
constexpr int RG_OUT = RG_LANES - 2;
constexpr int RG_ROWS = WV_LANES / RG_LANES;

// Tile order.  Workgroups go to the eight XCDs in turn (block b runs on XCD
// b mod 8), each with its own L2.  Consecutive groups of S tiles (the
// segments of a few neighbouring rows of one x_3 chunk) are dealt to the
// XCDs in turn, so the rows of a group share one L2 while all eight XCDs
// work through the same x_3 chunk at the same time.  The grid is padded to
// a multiple of 8 S; tiles at or beyond the count do nothing.
__device__ __forceinline__ int w3_tile(int S) {
  const int bid = blockIdx.x, slot = bid >> 3;
  return ((slot / S) * 8 + (bid & 7)) * S + slot % S;
}
static unsigned w3_grid(int64_t ntiles, int S) { return (unsigned)(8 * S * ((ntiles + 8 * S - 1) / (8 * S))); }

// DPP wavefront shifts: FROM_LEFT gives lane i the value of lane i-1,
// FROM_RIGHT the value of lane i+1 (zero where that lane does not exist).
constexpr int DPP_WAVE_SHL1 = 0x130;
constexpr int DPP_WAVE_SHR1 = 0x138;

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <typename T> __device__ __forceinline__ T fromL(T v) { return dpp<DPP_WAVE_SHR1>(v); }
template <typename T> __device__ __forceinline__ T fromR(T v) { return dpp<DPP_WAVE_SHL1>(v); }
template <typename T> __device__ __forceinline__ cx<T> fromL(cx<T> v) { return mk(fromL(v.re), fromL(v.im)); }
template <typename T> __device__ __forceinline__ cx<T> fromR(cx<T> v) { return mk(fromR(v.re), fromR(v.im)); }
// The same shifts inside lane groups of G lanes (G = 64: the whole
// wavefront; G = 16: DPP rows), zero at the group's edges.
constexpr int DPP_ROW_SHL1 = 0x101;
constexpr int DPP_ROW_SHR1 = 0x111;
template <int G, typename T> __device__ __forceinline__ T gL(T v) {
  return dpp<G == 64 ? DPP_WAVE_SHR1 : DPP_ROW_SHR1>(v);
}
template <int G, typename T> __device__ __forceinline__ T gR(T v) {
  return dpp<G == 64 ? DPP_WAVE_SHL1 : DPP_ROW_SHL1>(v);
}
template <int G, typename T> __device__ __forceinline__ cx<T> gL(cx<T> v) { return mk(gL<G>(v.re), gL<G>(v.im)); }
template <int G, typename T> __device__ __forceinline__ cx<T> gR(cx<T> v) { return mk(gR<G>(v.re), gR<G>(v.im)); }

// amp * (delta/width)^2, delta the distance into the absorbing layer at
// physical coordinate xp along an axis of physical length len.
template <typename T>
__device__ __forceinline__ T absorb(T xp, T len, T w, T iw, T amp) {
  T d = (w - xp > T(0) ? w - xp : T(0)) + (xp - (len - w) > T(0) ? xp - (len - w) : T(0));
  T r = d * iw;
  return amp * r * r;
}

// Buffer resources (raw, stride 0): the plane offset of the march goes into
// the scalar offset, the lane offsets stay fixed.  Offsets at or beyond the
// resource size read as zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* p, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0,
                                           (int)(bytes > 0x7fffffffll ? 0x7fffffffll : bytes), 0x00020000);
}
template <typename V> __device__ __forceinline__ V bload(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <> __device__ __forceinline__ float bload<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <> __device__ __forceinline__ double bload<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <> __device__ __forceinline__ cx<float> bload<cx<float>>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(cx<float>, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <> __device__ __forceinline__ cx<double> bload<cx<double>>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(cx<double>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
__device__ __forceinline__ void bstore(cx<float> v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r,
                                        voff, soff, 0);
}
__device__ __forceinline__ void bstore(cx<double> v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned, v), r,
                                         voff, soff, 0);
}

// Workgroup barrier for the LDS hand-off of the divergence terms: waits for
// this wave's LDS operations only, so buffer loads stay in flight.
__device__ __forceinline__ void lds_barrier_w3() {
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_s_barrier();
}

}  // namespace

template <typename T> struct W3Ctx {
  int n1, n2, n3, plane, c1, c2, z0, z1;
  bool inx, outlane;
  int roff[4];  // in-plane cell numbers of rows c-2 .. c+1 (clamped)
  bool rok[4];
  int offLc;    // cell left of (c1, c2) (clamped)
  __amdgpu_buffer_rsrc_t RX[4], RY[4], RB[4], RMU, RRHO, RKAP;
  T beta, omb, ih, ih2, cn, omega2;
  bool has_abl;
  T h, len1, len2, len3, abl_w, abl_iw, abl_amp, gam;
  const T* ablz;  // x_3 part of the absorbing layer per plane (centres, then lower faces)
  T gf;         // gamma (+alpha) + x_1 and x_2 parts of the layer at this wave's faces
  // fused restriction of the residual (restriction mode only)
  int role;     // 0: fine row 2J (stores coarse row J), 1: fine row 2J+1, 2: the u_2 rows of fine row 2J-1
  int Jc, Z0, Z1, nc1, nc2;  // coarse row, coarse planes [Z0, Z1) of the chunk, coarse cells along x_1, x_2
  int64_t cfs;               // coarse cells per field
  cx<T>* yc;                 // coarse vector of this right-hand side
  cx<T> (*RZ)[5][WV_LANES];  // LDS hand-off by coarse-plane parity: rows 2J+1 (u_1..u_3, p) and 2J-1 (u_2)
};

// Restriction along x_1 of a residual row held one fine face / cell per
// lane: the full weighting (1/4)[1 2 1] for u_1 (FN == 0), the pair mean
// otherwise; the result is meaningful at lanes holding an even c_1.
template <int FN, typename T>
__device__ __forceinline__ cx<T> rr_x1(cx<T> r) {
  if (FN == 0) return T(0.25) * (fromL(r) + fromR(r)) + T(0.5) * r;
  return T(0.5) * (r + fromR(r));
}

// x_2 step of the fused restriction and the store of coarse plane I3 of
// coarse row J by the waves of fine row 2J: u_2 takes (1/4)[1 2 1] over
// fine rows 2J-1, 2J, 2J+1, the other fields the pair mean of rows 2J and
// 2J+1.  Coarse faces on the domain boundary are written as zero.
template <int K, typename T>
__device__ __forceinline__ void rr_emit(const W3Ctx<T>& C, int I3, cx<T> rz, cx<T> rzp) {
  const int lane = threadIdx.x;
  const int par = I3 & 1;
  cx<T> v;
  if (K == 1) v = T(0.5) * rz + T(0.25) * (C.RZ[par][1][lane] + C.RZ[par][4][lane]);
  else v = T(0.5) * (rz + C.RZ[par][K][lane]);
  if ((lane & 1) == 0 && lane >= 2 && lane <= WV_LANES - 4 && C.c1 < C.n1) {
    const int I1 = C.c1 >> 1;
    const bool bnd = K == 0 ? I1 == 0 : (K == 1 ? C.Jc == 0 : I3 == 0);
    const int64_t o = ((int64_t)I3 * C.nc2 + C.Jc) * C.nc1 + I1;
    C.yc[K * C.cfs + o] = bnd ? czero<T>() : v;
    if (K == 0) C.yc[3 * C.cfs + o] = T(0.5) * (rzp + C.RZ[par][3][lane]);
  }
}

// Per-wavefront context of the march: tile coordinates, clamped row
// offsets, buffer resources, constants, gamma~ of this wavefront's faces.
// G: lanes per x_1 segment (64, or 16 with one x_2 row per group; c2 is
// then the lane's row, and rows at or beyond n_2 store nothing)
template <typename T, typename TI, bool RESID, int G = WV_LANES>
__device__ __forceinline__ void w3_setup(W3Ctx<T>& C, const LevelArgs<T>& L, const cx<TI>* __restrict__ x,
                                         const cx<T>* __restrict__ b, cx<T>* __restrict__ y, int c1o, int k, int c2,
                                         int tz, int zc, int s) {
  C.n1 = L.n[0]; C.n2 = L.n[1]; C.n3 = L.n[2];
  C.plane = C.n1 * C.n2;
  const int gl = (int)threadIdx.x & (G - 1);
  C.c1 = c1o + gl;
  C.c2 = c2;
  C.z0 = tz * zc;
  C.z1 = min(C.z0 + zc, C.n3);
  C.inx = C.c1 >= 0 && C.c1 < C.n1;
  C.outlane = gl >= 1 && gl <= G - 2 && C.inx && c2 < C.n2;
  const int cc1 = min(max(C.c1, 0), C.n1 - 1);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int rr = c2 - 2 + r;
    C.rok[r] = rr >= 0 && rr < C.n2;
    C.roff[r] = min(max(rr, 0), C.n2 - 1) * C.n1 + cc1;
  }
  C.offLc = min(max(c2, 0), C.n2 - 1) * C.n1 + max(cc1 - 1, 0);
  const int64_t fs = L.fs;
  const cx<TI>* xs = x + (int64_t)s * L.vs;
  cx<T>* ys = y + (int64_t)s * L.vs;
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    C.RX[f] = rsrc(xs + f * fs, fs * (int64_t)sizeof(cx<TI>));
    C.RY[f] = rsrc(ys + f * fs, fs * (int64_t)sizeof(cx<T>));
    C.RB[f] = RESID ? rsrc(b + (int64_t)s * L.vs + f * fs, fs * (int64_t)sizeof(cx<T>)) : C.RY[f];
  }
  C.RMU = rsrc(L.mu, fs * (int64_t)sizeof(T));
  C.RRHO = rsrc(L.rho, fs * (int64_t)sizeof(T));
  C.RKAP = rsrc(L.kap, fs * (int64_t)sizeof(T));
  C.beta = L.beta; C.omb = T(1) - L.beta;
  C.ih = L.ih; C.ih2 = L.ih * L.ih;
  C.cn = C.omb / T(6);
  C.omega2 = L.omega2;
  C.has_abl = L.abl_w > T(0) && L.abl_amp != T(0);
  C.h = L.h; C.len1 = C.n1 * L.h; C.len2 = C.n2 * L.h; C.len3 = C.n3 * L.h;
  C.gam = L.gam;
  C.abl_w = L.abl_w; C.abl_iw = L.abl_iw; C.abl_amp = L.abl_amp;
  C.ablz = L.ablz;
  // gamma~ at this wave's faces: x_1 / x_2 parts of the layer (the face of
  // u_k sits at a cell edge along x_k and at cell centres otherwise)
  C.gf = L.gam;
  if (C.has_abl) {
    const T hf = T(0.5);
    const T x1 = (k == 0 ? T(C.c1) : T(C.c1) + hf) * L.h;
    const T x2 = (k == 1 ? T(c2) : T(c2) + hf) * L.h;
    C.gf += absorb<T>(x1, C.n1 * L.h, L.abl_w, L.abl_iw, L.abl_amp) +
            absorb<T>(x2, C.n2 * L.h, L.abl_w, L.abl_iw, L.abl_amp);
  }
}

// RR (restriction mode, RESID true): the residual rows are restricted to
// the coarse level instead of stored; the march then takes its planes in
// (odd, even) pairs from 2 Z0 - 3, so that the residual of plane 2 Z0 - 1,
// which the x_3 full weighting of u_3 needs, is exact.
template <int K, typename T, typename TI, bool RESID, bool RR = false, int G = WV_LANES>
__device__ __forceinline__ void w3_march(const W3Ctx<T>& C, cx<T> (*DV)[3][WV_LANES]) {
  static_assert(G == WV_LANES || !RR, "the fused restriction marches whole wavefronts");
  constexpr int CB = (int)sizeof(cx<T>), CBI = (int)sizeof(cx<TI>), RBY = (int)sizeof(T);
  const T q = T(0.25), hf = T(0.5);
  const T beta = C.beta;
  const T oq = C.omb * q, oh = C.omb * hf;  // (1-beta)/4, (1-beta)/2 of the spread
  const int lane = threadIdx.x;
  const int n3 = C.n3;
  int vu[3], vi[3], vr[4];  // lane byte offsets: output/rhs fields, input fields, media
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    vu[r] = C.roff[r + 1] * CB;
    vi[r] = C.roff[r + 1] * CBI;
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) vr[r] = C.roff[r] * RBY;
  const int vrL = C.offLc * RBY;
  auto zcl = [&](int z) { return min(max(z, 0), n3 - 1) * C.plane; };
  // mask of u_{K+1} at row r (0: c-1, 1: c, 2: c+1) of plane z
  auto uok = [&](int r, int z) {
    bool ok = C.inx && C.rok[r + 1] && z >= 0 && z < n3;
    if (K == 0) ok = ok && C.c1 > 0;
    if (K == 1) ok = ok && C.c2 - 1 + r > 0;
    if (K == 2) ok = ok && z > 0;
    return ok;
  };

  // loads in flight for the next plane (input precision TI)
  cx<TI> nu[3];
  cx<TI> npm, npc;
  T nmu[3], nrho[4], nrhoL;
  T na3;  // x_3 part of gamma~ for plane z-1: a table entry fetched with the plane-z loads, as a
          // vector load, so no wait on the scalar cache stalls the LDS hand-off
  // kappa and b_p of plane z-1 for the p row (wavefront 0) are fetched with
  // the plane-z loads: loaded after the barrier in the step itself, waiting
  // for them would also wait for the whole next-plane prefetch (vector loads
  // complete in order), once per plane, and the barrier makes the other two
  // wavefronts wait with it.  float64 also fetches the b of this wavefront's
  // row a plane ahead (12-14 % faster at two waves per SIMD); float32 loads
  // it at the start of the step, before the prefetch, where it delays
  // nothing (fetched a plane ahead it gave no time and 7-20 % more traffic).
  constexpr bool PF = sizeof(T) == 8;
  constexpr bool PFP = true;
  T nkq = T(0);
  cx<T> nbp = czero<T>(), nbq = czero<T>();
  const __amdgpu_buffer_rsrc_t RABL = rsrc(C.ablz, C.has_abl ? 2 * n3 * RBY : 0);
  auto load_next = [&](int z) {
    na3 = bload<T>(RABL, 0, ((K == 2 ? n3 : 0) + min(max(z - 1, 0), n3 - 1)) * RBY);
    if (PF && RESID) nbq = bload<cx<T>>(C.RB[K], vu[1], zcl(z - 1) * CB);
    if (PFP && K == 0) {
      nkq = bload<T>(C.RKAP, vr[2], zcl(z - 1) * RBY);
      if (RESID) nbp = bload<cx<T>>(C.RB[3], vu[1], zcl(z - 1) * CB);
    }
    const int so = zcl(z) * CBI, sr = zcl(z) * RBY;
#pragma unroll
    for (int r = 0; r < 3; ++r) nu[r] = bload<cx<TI>>(C.RX[K], vi[r], so);
    npc = bload<cx<TI>>(C.RX[3], vi[1], so);
    if (K == 1) npm = bload<cx<TI>>(C.RX[3], vi[0], so);
    if (K == 1) {
      nmu[0] = bload<T>(C.RMU, vr[1], sr);
      nmu[1] = bload<T>(C.RMU, vr[2], sr);
    } else {
#pragma unroll
      for (int r = 0; r < 3; ++r) nmu[r] = bload<T>(C.RMU, vr[r + 1], sr);
    }
    if (K == 1) {
#pragma unroll
      for (int r = 0; r < 4; ++r) nrho[r] = bload<T>(C.RRHO, vr[r], sr);
    } else {
#pragma unroll
      for (int r = 1; r < 4; ++r) nrho[r] = bload<T>(C.RRHO, vr[r], sr);
    }
    if (K == 0) nrhoL = bload<T>(C.RRHO, vrL, sr);
  };

  // windows (plane t is the output plane); UA/UB and WA/WB are used
  // ping-pong: the step for plane t overwrites the plane t-1 half
  cx<T> UA[3], UB[3];   // u at rows c-1, c, c+1
  cx<T> WA, WB;         // rho_f u at row c
  cx<T> Y3b, F3, Wmp;   // Y_3 at (c, t); x_3 flux below plane t (times h^2); rho_f u at (c-1, t) + (c+1, t)
  cx<T> PA, PB, Pbm;    // p at (c, t-1) / (c, t) ping-pong; p at (c-1, t)
  T MA[3], MB[3];       // mu at rows c-1, c, c+1 (planes t-1 / t ping-pong)
  T rhob[3];            // rho at rows c-1, c, c+1 (plane t)
  // two warm-up planes, plus one more where the chunk starts on an odd plane:
  // the loop below takes planes in pairs, and anchoring the pairs to even
  // planes makes every plane go through the same copy of the step whatever
  // the chunk length, so all chunk lengths give the same bits
  const int t0 = RR ? C.z0 - 3 : C.z0 - 2 - (C.z0 & 1);
  // restriction mode: x_1-restricted residual at planes t-1, t-2 (p row:
  // rxp1), and the x_1/x_3-restricted values of the last odd plane kept by
  // the waves of row 2J until the x_2 step
  cx<T> rx1 = czero<T>(), rx2 = czero<T>(), rz = czero<T>(), rxp1 = czero<T>(), rzp = czero<T>();
#pragma unroll
  for (int r = 0; r < 3; ++r) UA[r] = UB[r] = czero<T>();
  WA = WB = Y3b = F3 = Wmp = czero<T>();
  PA = PB = Pbm = czero<T>();
  {
    const int sr = zcl(t0) * RBY;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      MA[r] = MB[r] = bload<T>(C.RMU, vr[r + 1], sr);
      rhob[r] = bload<T>(C.RRHO, vr[r + 1], sr);
    }
  }
  load_next(t0 + 1);

  auto step = [&](int t, bool odd, cx<T>(&UO)[3], cx<T>(&UC)[3], cx<T>& WO, cx<T>& WC, T(&MO)[3], T(&MC)[3],
                  cx<T>& PO, cx<T>& PC) {
    const int tn = t + 1;
    const bool zok = tn >= 0 && tn < n3;
    const int sc = zcl(t) * CB;
    cx<T> bq = nbq;
    if (!PF && RESID) bq = bload<cx<T>>(C.RB[K], vu[1], sc);
    // plane t+1: masked u, p and the media this component uses
    cx<T> Un[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) Un[r] = uok(r, tn) ? mk(T(nu[r].re), T(nu[r].im)) : czero<T>();
    const cx<T> Pnc = (C.inx && zok) ? mk(T(npc.re), T(npc.im)) : czero<T>();
    const cx<T> Pnm = (K == 1 && C.inx && C.rok[1] && zok) ? mk(T(npm.re), T(npm.im)) : czero<T>();
    T mun[3], rhon[3], rf[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      mun[r] = nmu[r];
      rhon[r] = nrho[r + 1];
    }
    // face means of rho for this component at rows c-1, c, c+1
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      if (K == 0) rf[r] = hf * ((r == 1 ? nrhoL : gL<G>(rhon[r])) + rhon[r]);
      if (K == 1) rf[r] = hf * (nrho[r] + rhon[r]);
      if (K == 2) rf[r] = hf * (rhob[r] + rhon[r]);
    }
    const T a3 = na3;  // x_3 part of gamma~ at this plane's faces
    const T kqp = nkq;
    const cx<T> bpp = nbp;
    load_next(t + 2);
    const cx<T> Wn = rf[1] * Un[1];
    const cx<T> Wmpn = rf[0] * Un[0] + rf[2] * Un[2];
    // Y_3(t+1) = beta u + (1-beta) A_1 A_2 u at row c
    const cx<T> V = q * (Un[0] + Un[2]) + hf * Un[1];
    const cx<T> Y3n = beta * Un[1] + oq * (gL<G>(V) + gR<G>(V)) + oh * V;
    // A_3 u(t) at rows c-1, c, c+1; Y_1(t) (row c) and Y_2(t) (three rows)
    cx<T> Z[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) Z[r] = q * (UO[r] + Un[r]) + hf * UC[r];
    const cx<T> y1 = beta * UC[1] + oq * (Z[0] + Z[2]) + oh * Z[1];
    cx<T> y2[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) y2[r] = beta * UC[r] + oq * (gL<G>(Z[r]) + gR<G>(Z[r])) + oh * Z[r];
    const cx<T> d1lo = y1 - gL<G>(y1);
    const cx<T> d1hi = gR<G>(d1lo);
    const cx<T> d2lo = y2[1] - y2[0], d2hi = y2[2] - y2[1];
    cx<T> acc, F3n, dv;
    if (K == 0) {
      // x_1 flux with cell mu; x_2 / x_3 fluxes with mu averaged over the
      // four cells around the edge (pairs along x_1 first)
      T MXb[3], MXn1;
#pragma unroll
      for (int r = 0; r < 3; ++r) MXb[r] = hf * (gL<G>(MC[r]) + MC[r]);
      MXn1 = hf * (gL<G>(mun[1]) + mun[1]);
      acc = gL<G>(MC[1]) * d1lo - MC[1] * d1hi;
      acc += (hf * (MXb[0] + MXb[1])) * d2lo - (hf * (MXb[1] + MXb[2])) * d2hi;
      F3n = (hf * (MXb[1] + MXn1)) * (Y3n - Y3b);
      dv = d1hi;
    } else if (K == 1) {
      const T MYb = hf * (MC[0] + MC[1]), MYn = hf * (mun[0] + mun[1]);
      acc = MC[0] * d2lo - MC[1] * d2hi;
      acc += (hf * (gL<G>(MYb) + MYb)) * d1lo - (hf * (MYb + gR<G>(MYb))) * d1hi;
      F3n = (hf * (MYb + MYn)) * (Y3n - Y3b);
      dv = d2hi;
    } else {
      const T MZm = hf * (MO[0] + MC[0]), MZc = hf * (MO[1] + MC[1]), MZp = hf * (MO[2] + MC[2]);
      acc = (hf * (gL<G>(MZc) + MZc)) * d1lo - (hf * (MZc + gR<G>(MZc))) * d1hi;
      acc += (hf * (MZm + MZc)) * d2lo - (hf * (MZc + MZp)) * d2hi;
      F3n = MC[1] * (Y3n - Y3b);
      dv = Y3n - Y3b;
    }
    acc = C.ih2 * (acc + F3 - F3n);
    // spread mass with the attenuation of the output face
    const cx<T> nb = gL<G>(WC) + gR<G>(WC) + Wmp + WO + Wn;
    const cx<T> sm = beta * WC + C.cn * nb;
    acc -= mk(C.omega2, -C.omega2 * (C.gf + a3)) * sm;
    // coupling with p: the cell above the face minus the cell below
    if (K == 0) acc += C.ih * (PC - gL<G>(PC));
    if (K == 1) acc += C.ih * (PC - Pbm);
    if (K == 2) acc += C.ih * (PC - PO);
    const bool emit = !RR && C.outlane && t >= C.z0;
    if (RR) {
      // every lane takes part in the lane shifts; boundary faces feed only
      // coarse boundary faces, which are written as zero
      const cx<T> rx = rr_x1<K>(bq - acc);
      if (odd) {
        const cx<T> v = K == 2 ? q * (rx2 + rx) + hf * rx1 : hf * (rx1 + rx);
        if (C.role != 0) C.RZ[(t >> 1) & 1][C.role == 1 ? K : 4][lane] = v;
        rz = v;  // used by row 2J only
      }
      rx2 = rx1;
      rx1 = rx;
    } else if (emit) {
      const bool face = K == 0 ? C.c1 > 0 : (K == 1 ? C.c2 > 0 : t > 0);
      cx<T> v = face ? acc : czero<T>();
      if (RESID && face) v = bq - v;
      bstore(v, C.RY[K], vu[1], sc);
    }
    // divergence term of the p row of cell (c1, c2, t)
    DV[t & 1][K][lane] = C.ih * dv;
    // advance the windows: plane t+1 replaces plane t-1
    F3 = F3n;
    Y3b = Y3n;
    WO = Wn;
    Wmp = Wmpn;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      UO[r] = Un[r];
      MO[r] = mun[r];
      rhob[r] = rhon[r];
    }
    PO = Pnc;
    Pbm = Pnm;
    lds_barrier_w3();
    if (K == 0 && (emit || (RR && C.role != 2))) {
      cx<T> vp = C.ih * dv + DV[t & 1][1][lane] + DV[t & 1][2][lane];
      const T kq = PFP ? kqp : bload<T>(C.RKAP, vr[2], zcl(t) * RBY);
      vp += kq * PC;
      if (RESID) vp = (PFP ? bpp : bload<cx<T>>(C.RB[3], vu[1], sc)) - vp;
      if (RR) {
        const cx<T> rxp = rr_x1<3>(vp);
        if (odd) {
          const cx<T> v = hf * (rxp1 + rxp);
          if (C.role != 0) C.RZ[(t >> 1) & 1][3][lane] = v;
          rzp = v;
        }
        rxp1 = rxp;
      } else {
        bstore(vp, C.RY[3], vu[1], sc);
      }
    }
    // coarse plane (t - 2) / 2, handed over before this plane's barrier
    if (RR && !odd && C.role == 0 && t >= 2 * C.Z0 + 2) rr_emit<K>(C, (t >> 1) - 1, rz, rzp);
  };

  for (int t = t0; t < C.z1; t += 2) {
    step(t, RR, UA, UB, WA, WB, MA, MB, PA, PB);
    if (t + 1 < C.z1) step(t + 1, !RR, UB, UA, WB, WA, MB, MA, PB, PA);
  }
  if (RR) {
    // the last odd plane of the chunk: its coarse plane Z1 - 1
    lds_barrier_w3();
    if (C.role == 0) rr_emit<K>(C, C.Z1 - 1, rz, rzp);
  }
}

// Adjoint (conjugate transpose) rows, same march.  For H^H the spread acts
// after the flux: along each axis l the flux G_l = A_e(mu) D_l u (cell mu
// when l = k) is formed at every flux point, spread by S_l over the other
// two axes, and differenced along l.  The mass takes conj(omega^2 (1 - i
// gamma~)) at each of the seven points and rho_f at the output face; the
// coupling applies S_k to p before the difference; the p row is kappa p
// plus the plain differences of the u_k.  Wavefront K keeps: u at planes t
// and t+1 (rows c-1..c+1); A_2 G_1 at planes t-1, t; A_1 G_2 at the two
// flux rows, planes t-1, t; the spread x_3 flux below plane t; the
// attenuated u of the mass at (c, t-1), (c, t); the partial spreads of p.
// RR: restriction mode as in w3_march (one step per plane here, so the
// plane parity is a run-time value).
template <int K, typename T, bool RESID, bool RR = false, int G = WV_LANES>
__device__ __forceinline__ void w3_march_adj(const W3Ctx<T>& C, cx<T> (*DV)[3][WV_LANES]) {
  static_assert(G == WV_LANES || !RR, "the fused restriction marches whole wavefronts");
  constexpr int CB = (int)sizeof(cx<T>), RBY = (int)sizeof(T);
  const T q = T(0.25), hf = T(0.5);
  const T beta = C.beta;
  const T oq = C.omb * q, oh = C.omb * hf;  // (1-beta)/4, (1-beta)/2 of the spread
  const int lane = threadIdx.x;
  const int n3 = C.n3;
  int vu[3], vr[4], vl[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) vu[r] = C.roff[r + 1] * CB;
#pragma unroll
  for (int r = 0; r < 4; ++r) vr[r] = C.roff[r] * RBY;
  // the u_1 fluxes along x_2 and x_3 at lane 0 feed lane 1 through the
  // spread, and their edge means need mu one cell to the left: load it
  // rather than take it from the neighbouring lane
  const int lshift = C.c1 > 0 && C.c1 <= C.n1 - 1 ? 1 : 0;
#pragma unroll
  for (int r = 0; r < 3; ++r) vl[r] = (C.roff[r + 1] - lshift) * RBY;
  auto zcl = [&](int z) { return min(max(z, 0), n3 - 1) * C.plane; };
  auto uok = [&](int r, int z) {
    bool ok = C.inx && C.rok[r + 1] && z >= 0 && z < n3;
    if (K == 0) ok = ok && C.c1 > 0;
    if (K == 1) ok = ok && C.c2 - 1 + r > 0;
    if (K == 2) ok = ok && z > 0;
    return ok;
  };
  auto pok = [&](int r, int z) { return C.inx && C.rok[r + 1] && z >= 0 && z < n3; };
  // attenuation gamma~ at this component's faces: x_1 / x_2 parts per row
  // (rows c-1, c, c+1) and the x_3 part per plane
  T gxy[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    gxy[r] = C.gam;
    if (C.has_abl) {
      const T x1 = (K == 0 ? T(C.c1) : T(C.c1) + hf) * C.h;
      const T x2 = (K == 1 ? T(C.c2 - 1 + r) : T(C.c2 - 1 + r) + hf) * C.h;
      gxy[r] += absorb<T>(x1, C.len1, C.abl_w, C.abl_iw, C.abl_amp) +
                absorb<T>(x2, C.len2, C.abl_w, C.abl_iw, C.abl_amp);
    }
  }
  auto a3of = [&](int z) {  // x_3 part of gamma~ at plane z's faces (table entry)
    return C.has_abl ? C.ablz[(K == 2 ? n3 : 0) + min(max(z, 0), n3 - 1)] : T(0);
  };
  auto att = [&](T g, cx<T> u) { return mk(u.re - g * u.im, u.im + g * u.re); };  // (1 + i g) u
  auto A1 = [&](cx<T> v) { return q * (gL<G>(v) + gR<G>(v)) + hf * v; };

  // loads in flight for the next plane
  cx<T> nu[3], np[3];
  T nmu[4], nrho[2], nmuL[3];
  T na3;  // x_3 part of gamma~ for plane z (table entry, loaded with plane z)
  // b of this wavefront's row and, for the p row (wavefront 0), kappa and
  // b_p of plane z-1, fetched with the plane-z loads
  T nkq = T(0);
  cx<T> nbp = czero<T>(), nbq = czero<T>();
  const __amdgpu_buffer_rsrc_t RABL = rsrc(C.ablz, C.has_abl ? 2 * n3 * RBY : 0);
  auto load_next = [&](int z) {
    na3 = bload<T>(RABL, 0, ((K == 2 ? n3 : 0) + min(max(z, 0), n3 - 1)) * RBY);
    if (RESID) nbq = bload<cx<T>>(C.RB[K], vu[1], zcl(z - 1) * CB);
    if (K == 0) {
      nkq = bload<T>(C.RKAP, vr[2], zcl(z - 1) * RBY);
      if (RESID) nbp = bload<cx<T>>(C.RB[3], vu[1], zcl(z - 1) * CB);
    }
    const int so = zcl(z) * CB, sr = zcl(z) * RBY;
#pragma unroll
    for (int r = 0; r < 3; ++r) nu[r] = bload<cx<T>>(C.RX[K], vu[r], so);
#pragma unroll
    for (int r = 0; r < 3; ++r)
      if (K != 1 || r < 2) np[r] = bload<cx<T>>(C.RX[3], vu[r], so);
    if (K == 1) {
#pragma unroll
      for (int r = 0; r < 4; ++r) nmu[r] = bload<T>(C.RMU, vr[r], sr);
      nrho[0] = bload<T>(C.RRHO, vr[1], sr);
      nrho[1] = bload<T>(C.RRHO, vr[2], sr);
    } else {
#pragma unroll
      for (int r = 0; r < 3; ++r) nmu[r + 1] = bload<T>(C.RMU, vr[r + 1], sr);
      nrho[1] = bload<T>(C.RRHO, vr[2], sr);
    }
    if (K == 0) {
#pragma unroll
      for (int r = 0; r < 3; ++r) nmuL[r] = bload<T>(C.RMU, vl[r], sr);
    }
  };

  // windows
  cx<T> UC[3];                 // u at (rows c-1..c+1, plane t)
  cx<T> X1a, X1b, G1b;         // A_2 G_1 at t-1, t; G_1 at (c, t)
  cx<T> Q2la, Q2lb, Q2ha, Q2hb, G2lb, G2hb;  // A_1 G_2 at the lower / upper flux row, t-1 and t; G_2 at t
  cx<T> SG3;                   // spread x_3 flux through the face below plane t
  cx<T> Wa, Wb;                // attenuated u at (c, t-1), (c, t)
  cx<T> Pa0, Pb0, Pa1, Pb1, Pc0, Pc1;  // partial spreads of p (meaning depends on K)
  T mub[4];                    // mu at plane t (rows c-2..c+1; K != 1 uses 1..3)
  T mubL[3];                   // K == 0: mu one cell to the left at plane t (rows c-1..c+1)
  T rhoa, rhob0, rhob1;        // rho: (c, t-1); plane t rows (K == 1: c-1, c; else c)
  T a3a, a3b;                  // x_3 part of gamma~ at planes t-1, t
  const int t0 = RR ? C.z0 - 3 : C.z0 - 2;
  cx<T> rx1 = czero<T>(), rx2 = czero<T>(), rz = czero<T>(), rxp1 = czero<T>(), rzp = czero<T>();
#pragma unroll
  for (int r = 0; r < 3; ++r) UC[r] = czero<T>();
  X1a = X1b = G1b = Q2la = Q2lb = Q2ha = Q2hb = G2lb = G2hb = SG3 = Wa = Wb = czero<T>();
  Pa0 = Pb0 = Pa1 = Pb1 = Pc0 = Pc1 = czero<T>();
  {
    const int sr = zcl(t0) * RBY;
#pragma unroll
    for (int r = 0; r < 4; ++r) mub[r] = bload<T>(C.RMU, vr[r], sr);
#pragma unroll
    for (int r = 0; r < 3; ++r) mubL[r] = K == 0 ? bload<T>(C.RMU, vl[r], sr) : T(0);
    rhob0 = bload<T>(C.RRHO, vr[K == 1 ? 1 : 2], sr);
    rhob1 = bload<T>(C.RRHO, vr[2], sr);
    rhoa = rhob1;
  }
  a3a = a3b = a3of(t0);
  load_next(t0 + 1);

  for (int t = t0; t < C.z1; ++t) {
    const int tn = t + 1;
    const int sc = zcl(t) * CB;
    // plane t+1, masked
    cx<T> Un[3], Pn[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      Un[r] = uok(r, tn) ? nu[r] : czero<T>();
      Pn[r] = (pok(r, tn) && (K != 1 || r < 2)) ? np[r] : czero<T>();
    }
    T mun[4], munL[3], rhon0, rhon1;
#pragma unroll
    for (int r = 0; r < 4; ++r) mun[r] = (K == 1 || r > 0) ? nmu[r] : T(0);
#pragma unroll
    for (int r = 0; r < 3; ++r) munL[r] = K == 0 ? nmuL[r] : T(0);
    rhon0 = K == 1 ? nrho[0] : nrho[1];
    rhon1 = nrho[1];
    const T a3n = na3;
    const T kq = nkq;
    const cx<T> bp = nbp, bq = nbq;
    load_next(t + 2);

    // edge/cell mu of this component's fluxes at plane t+1 (and between t, t+1)
    T mu1[3], mu2l, mu2h, mu3[3];
    if (K == 0) {
      T MXn[3], MXb[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        MXn[r] = hf * (munL[r] + mun[r + 1]);
        MXb[r] = hf * (mubL[r] + mub[r + 1]);
        mu1[r] = mun[r + 1];                 // cell mu (flux along x_1 of u_1)
        mu3[r] = hf * (MXb[r] + MXn[r]);     // edges between planes t, t+1
      }
      mu2l = hf * (MXn[0] + MXn[1]);
      mu2h = hf * (MXn[1] + MXn[2]);
    } else if (K == 1) {
      T MYn[3], MYb[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        MYn[r] = hf * (mun[r] + mun[r + 1]);
        MYb[r] = hf * (mub[r] + mub[r + 1]);
        mu1[r] = hf * (gL<G>(MYn[r]) + MYn[r]);
        mu3[r] = hf * (MYb[r] + MYn[r]);
      }
      mu2l = mun[1];  // cell mu of rows c-1 and c (flux along x_2 of u_2)
      mu2h = mun[2];
    } else {
      T MZn[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        MZn[r] = hf * (mub[r + 1] + mun[r + 1]);
        mu1[r] = hf * (gL<G>(MZn[r]) + MZn[r]);
        mu3[r] = mub[r + 1];  // cell mu of plane t (flux along x_3 of u_3)
      }
      mu2l = hf * (MZn[0] + MZn[1]);
      mu2h = hf * (MZn[1] + MZn[2]);
    }
    // flux along x_1 at plane t+1 (lane x: cell x for u_1, edge x otherwise)
    cx<T> G1n[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) G1n[r] = mu1[r] * (K == 0 ? gR<G>(Un[r]) - Un[r] : Un[r] - gL<G>(Un[r]));
    const cx<T> X1n = q * (G1n[0] + G1n[2]) + hf * G1n[1];
    const cx<T> SG1 = beta * G1b + oq * (X1a + X1n) + oh * X1b;
    cx<T> acc = K == 0 ? gL<G>(SG1) - SG1 : SG1 - gR<G>(SG1);
    // flux along x_2 at the lower / upper flux row, plane t+1
    const cx<T> G2ln = mu2l * (Un[1] - Un[0]), G2hn = mu2h * (Un[2] - Un[1]);
    const cx<T> Q2ln = A1(G2ln), Q2hn = A1(G2hn);
    const cx<T> SG2l = beta * G2lb + oq * (Q2la + Q2ln) + oh * Q2lb;
    const cx<T> SG2h = beta * G2hb + oq * (Q2ha + Q2hn) + oh * Q2hb;
    acc += SG2l - SG2h;
    // flux along x_3 through the face between planes t and t+1
    cx<T> G3[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) G3[r] = mu3[r] * (Un[r] - UC[r]);
    const cx<T> V3 = q * (G3[0] + G3[2]) + hf * G3[1];
    const cx<T> SG3n = beta * G3[1] + oq * (gL<G>(V3) + gR<G>(V3)) + oh * V3;
    acc += SG3 - SG3n;
    acc = C.ih2 * acc;
    // adjoint spread mass: rho_f of the output face times the spread of
    // (1 + i gamma~) u over the seven points
    const cx<T> Wn = att(gxy[1] + a3n, Un[1]);
    const cx<T> nb = gL<G>(Wb) + gR<G>(Wb) + att(gxy[0] + a3b, UC[0]) + att(gxy[2] + a3b, UC[2]) + Wa + Wn;
    const cx<T> sm = beta * Wb + C.cn * nb;
    T rfP;
    if (K == 0) rfP = hf * (gL<G>(rhob1) + rhob1);
    else if (K == 1) rfP = hf * (rhob0 + rhob1);
    else rfP = hf * (rhoa + rhob1);
    acc -= (C.omega2 * rfP) * sm;
    // coupling: S_k p at the cells below and above the face, differenced
    cx<T> dv;
    if (K == 0) {
      const cx<T> A2n = q * (Pn[0] + Pn[2]) + hf * Pn[1];
      const cx<T> SP = beta * Pc0 + oq * (Pa0 + A2n) + oh * Pb0;
      acc += C.ih * (gL<G>(SP) - SP);
      dv = UC[1] - gR<G>(UC[1]);
      Pa0 = Pb0; Pb0 = A2n; Pc1 = Pc0; Pc0 = Pn[1];  // Pc1: p(c, t) for the p row
    } else if (K == 1) {
      const cx<T> A1m = A1(Pn[0]), A1c = A1(Pn[1]);
      const cx<T> SPm = beta * Pc0 + oq * (Pa0 + A1m) + oh * Pb0;
      const cx<T> SPc = beta * Pc1 + oq * (Pa1 + A1c) + oh * Pb1;
      acc += C.ih * (SPm - SPc);
      dv = UC[1] - UC[2];
      Pa0 = Pb0; Pb0 = A1m; Pa1 = Pb1; Pb1 = A1c; Pc0 = Pn[0]; Pc1 = Pn[1];
    } else {
      const cx<T> V = q * (Pn[0] + Pn[2]) + hf * Pn[1];
      const cx<T> SPn = beta * Pn[1] + oq * (gL<G>(V) + gR<G>(V)) + oh * V;
      acc += C.ih * (Pa0 - Pb0);
      dv = UC[1] - Un[1];
      Pa0 = Pb0; Pb0 = SPn;
    }
    const bool emit = !RR && C.outlane && t >= C.z0;
    const bool odd = t & 1;
    if (RR) {
      const cx<T> rx = rr_x1<K>(bq - acc);
      if (odd) {
        const cx<T> v = K == 2 ? q * (rx2 + rx) + hf * rx1 : hf * (rx1 + rx);
        if (C.role != 0) C.RZ[(t >> 1) & 1][C.role == 1 ? K : 4][lane] = v;
        rz = v;  // used by row 2J only
      }
      rx2 = rx1;
      rx1 = rx;
    } else if (emit) {
      const bool face = K == 0 ? C.c1 > 0 : (K == 1 ? C.c2 > 0 : t > 0);
      cx<T> v = face ? acc : czero<T>();
      if (RESID && face) v = bq - v;
      bstore(v, C.RY[K], vu[1], sc);
    }
    DV[t & 1][K][lane] = C.ih * dv;
    // advance the windows
    X1a = X1b; X1b = X1n; G1b = G1n[1];
    Q2la = Q2lb; Q2lb = Q2ln; Q2ha = Q2hb; Q2hb = Q2hn; G2lb = G2ln; G2hb = G2hn;
    SG3 = SG3n;
    Wa = Wb; Wb = Wn;
#pragma unroll
    for (int r = 0; r < 3; ++r) UC[r] = Un[r];
#pragma unroll
    for (int r = 0; r < 4; ++r) mub[r] = mun[r];
#pragma unroll
    for (int r = 0; r < 3; ++r) mubL[r] = munL[r];
    rhoa = rhob1; rhob0 = rhon0; rhob1 = rhon1;
    a3a = a3b; a3b = a3n;
    lds_barrier_w3();
    if (K == 0 && (emit || (RR && C.role != 2))) {
      // p row of cell (c1, c2, t): kappa p + the three differences
      cx<T> vp = DV[t & 1][0][lane] + DV[t & 1][1][lane] + DV[t & 1][2][lane];
      vp += kq * Pc1;
      if (RESID) vp = bp - vp;
      if (RR) {
        const cx<T> rxp = rr_x1<3>(vp);
        if (odd) {
          const cx<T> v = hf * (rxp1 + rxp);
          if (C.role != 0) C.RZ[(t >> 1) & 1][3][lane] = v;
          rzp = v;
        }
        rxp1 = rxp;
      } else {
        bstore(vp, C.RY[3], vu[1], sc);
      }
    }
    if (RR && !odd && C.role == 0 && t >= 2 * C.Z0 + 2) rr_emit<K>(C, (t >> 1) - 1, rz, rzp);
  }
  if (RR) {
    lds_barrier_w3();
    if (C.role == 0) rr_emit<K>(C, C.Z1 - 1, rz, rzp);
  }
  (void)a3a;
}

template <typename T, bool RESID>
__global__ void __launch_bounds__(WV_LANES * 3)
k_apply3d_w3_adj(LevelArgs<T> L, const cx<T>* __restrict__ x, const cx<T>* __restrict__ b, cx<T>* __restrict__ y,
                 int nfull, int nrem, int nzc, int zc, int ntiles) {
  // tiles as in k_apply3d_w3
  __shared__ cx<T> DV[2][3][WV_LANES];
  const int gs = RG_ROWS * nfull + nrem;
  const int tile = w3_tile(gs);
  if (tile >= ntiles) return;  // whole workgroup
  const int per_chunk = (L.n[1] + RG_ROWS - 1) / RG_ROWS * gs;
  int rest = tile;
  const int in = rest % per_chunk; rest /= per_chunk;
  const int tz = rest % nzc; rest /= nzc;
  const int s = rest;
  const int g = in / gs, j = in - g * gs;
  W3Ctx<T> C;
  const int k = threadIdx.y;
  if (j < RG_ROWS * nfull) {
    const int tx = j % nfull, c2 = g * RG_ROWS + j / nfull;
    if (c2 >= L.n[1]) return;  // whole workgroup
    w3_setup<T, T, RESID>(C, L, x, b, y, tx * WV_OUT - 1, k, c2, tz, zc, s);
    if (k == 0) w3_march_adj<0, T, RESID>(C, DV);
    else if (k == 1) w3_march_adj<1, T, RESID>(C, DV);
    else w3_march_adj<2, T, RESID>(C, DV);
  } else {
    const int c2 = g * RG_ROWS + (int)(threadIdx.x / RG_LANES);
    w3_setup<T, T, RESID, RG_LANES>(C, L, x, b, y, nfull * WV_OUT - 1, k, c2, tz, zc, s);
    if (k == 0) w3_march_adj<0, T, RESID, false, RG_LANES>(C, DV);
    else if (k == 1) w3_march_adj<1, T, RESID, false, RG_LANES>(C, DV);
    else w3_march_adj<2, T, RESID, false, RG_LANES>(C, DV);
  }
}

// Tiles per (x_3 chunk, rhs), in groups of RG_ROWS rows: the nfull 62-wide
// segments of each row of the group (x_1 fastest), then, when nrem is set,
// one tile for the last n_1 - 62 nfull (<= RG_OUT) cells of the group's rows,
// right after the segments whose cache lines it shares.  Tiles of rows beyond
// n_2 (last group) do nothing.
template <typename T, typename TI, bool RESID>
__global__ void __launch_bounds__(WV_LANES * 3)
k_apply3d_w3(LevelArgs<T> L, const cx<TI>* __restrict__ x, const cx<T>* __restrict__ b, cx<T>* __restrict__ y,
             int nfull, int nrem, int nzc, int zc, int ntiles) {
  __shared__ cx<T> DV[2][3][WV_LANES];
  const int gs = RG_ROWS * nfull + nrem;  // tiles per group of rows
  const int tile = w3_tile(gs);
  if (tile >= ntiles) return;  // whole workgroup
  const int per_chunk = (L.n[1] + RG_ROWS - 1) / RG_ROWS * gs;
  int rest = tile;
  const int in = rest % per_chunk; rest /= per_chunk;
  const int tz = rest % nzc; rest /= nzc;
  const int s = rest;
  const int g = in / gs, j = in - g * gs;
  W3Ctx<T> C;
  const int k = threadIdx.y;
  if (j < RG_ROWS * nfull) {
    const int tx = j % nfull, c2 = g * RG_ROWS + j / nfull;
    if (c2 >= L.n[1]) return;  // whole workgroup
    w3_setup<T, TI, RESID>(C, L, x, b, y, tx * WV_OUT - 1, k, c2, tz, zc, s);
    if (k == 0) w3_march<0, T, TI, RESID>(C, DV);
    else if (k == 1) w3_march<1, T, TI, RESID>(C, DV);
    else w3_march<2, T, TI, RESID>(C, DV);
  } else {
    const int c2 = g * RG_ROWS + (int)(threadIdx.x / RG_LANES);
    w3_setup<T, TI, RESID, RG_LANES>(C, L, x, b, y, nfull * WV_OUT - 1, k, c2, tz, zc, s);
    if (k == 0) w3_march<0, T, TI, RESID, false, RG_LANES>(C, DV);
    else if (k == 1) w3_march<1, T, TI, RESID, false, RG_LANES>(C, DV);
    else w3_march<2, T, TI, RESID, false, RG_LANES>(C, DV);
  }
}

// Residual + restriction, rc = R (b - H_s x) (ADJ: H_s^H): a workgroup of
// seven wavefronts for coarse row J of a 60-wide x_1 segment (fine cells
// c_1 = 60 tx - 2 + lane; lanes 1 and 62 are exact residual rows used by the
// full weighting, 0 and 63 halo) and a chunk of coarse planes.  Waves 0-2
// march fine row 2J (components u_1..u_3; wave 0 also the p row), waves 3-5
// row 2J+1, wave 6 the u_2 rows of row 2J-1.  Each restricts its residual
// along x_1 (lane shifts) and x_3 (register window); rows 2J+1 and 2J-1 hand
// theirs to row 2J through LDS, which does the x_2 step and the store.
template <typename T, bool ADJ>
__global__ void __launch_bounds__(WV_LANES * 7)
k_restrict_resid3d_w3(LevelArgs<T> L, LevelArgs<T> Lc, const cx<T>* __restrict__ x, const cx<T>* __restrict__ b,
                      cx<T>* __restrict__ yc, int tiles_x, int nzc, int zc, int ntiles) {
  __shared__ cx<T> DV[3][2][3][WV_LANES];  // per fine row (2J, 2J+1; unused third for wave 6)
  __shared__ cx<T> RZ[2][5][WV_LANES];
  const int tile = w3_tile(2 * tiles_x);  // groups of two coarse (four fine) rows
  if (tile >= ntiles) return;  // whole workgroup
  int rest = tile;
  const int tx = rest % tiles_x; rest /= tiles_x;
  const int J = rest % Lc.n[1]; rest /= Lc.n[1];
  const int tz = rest % nzc; rest /= nzc;
  const int s = rest;
  // the wave's index, as a wave-uniform (scalar) value: the role branches
  // below are then scalar branches
  const int wy = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
  const int role = wy < 3 ? 0 : (wy < 6 ? 1 : 2);
  const int k = wy < 6 ? wy % 3 : 1;
  const int c2 = 2 * J + (role == 1 ? 1 : (role == 2 ? -1 : 0));
  W3Ctx<T> C;
  // (the fine-level y resources are never stored through in this mode)
  w3_setup<T, T, true>(C, L, x, b, const_cast<cx<T>*>(b), tx * (WV_OUT - 2) - 2, k, c2, 0, 1, s);
  C.role = role;
  C.Jc = J;
  C.nc1 = Lc.n[0];
  C.nc2 = Lc.n[1];
  C.cfs = Lc.fs;
  C.yc = yc + (int64_t)s * Lc.vs;
  C.RZ = RZ;
  C.Z0 = tz * zc;
  C.Z1 = min(C.Z0 + zc, Lc.n[2]);
  C.z0 = 2 * C.Z0;
  C.z1 = 2 * C.Z1;
  cx<T>(*dv)[3][WV_LANES] = DV[role];
  if (ADJ) {
    if (k == 0) w3_march_adj<0, T, true, true>(C, dv);
    else if (k == 1) w3_march_adj<1, T, true, true>(C, dv);
    else w3_march_adj<2, T, true, true>(C, dv);
  } else {
    if (k == 0) w3_march<0, T, T, true, true>(C, dv);
    else if (k == 1) w3_march<1, T, T, true, true>(C, dv);
    else w3_march<2, T, T, true, true>(C, dv);
  }
}

// x_3 chunk length: zc < 0 asks for exactly -zc planes (the autotuner's
// candidates); otherwise zc (default 32) shortened so that at least ~8192
// workgroups are in flight on small grids
static int w3_chunk(const int* n, int64_t cols_per_rhs, int nrhs, int zc) {
  if (zc < 0) return -zc < n[2] ? -zc : n[2];
  if (zc == 0) zc = 32;
  const int64_t cols = cols_per_rhs * nrhs;
  const int64_t want = (int64_t)n[2] * cols / 8192;
  if (want < zc) zc = (int)(want < 4 ? 4 : want);
  if (zc > n[2]) zc = n[2];
  return zc;
}

template <typename T, typename TI>
int launch_apply3d_w3(const LevelArgs<T>& L, const void* x, const void* b, void* y, int nrhs, int zc,
                      hipStream_t st) {
  if (L.fs * (int64_t)sizeof(cx<T>) > (int64_t)0x7fffffff) return (int)hipErrorInvalidValue;
  // full 62-wide segments; a remainder of at most RG_OUT cells goes to
  // 16-lane row groups, a longer one to one more full segment
  int nfull = L.n[0] / WV_OUT, nrem = 0;
  const int rem = L.n[0] - nfull * WV_OUT;
  if (rem > RG_OUT) ++nfull;
  else if (rem > 0) nrem = 1;
  const int64_t per_chunk = (int64_t)(L.n[1] + RG_ROWS - 1) / RG_ROWS * (RG_ROWS * nfull + nrem);
  zc = w3_chunk(L.n, per_chunk, nrhs, zc);
  const int nzc = (L.n[2] + zc - 1) / zc;
  const int64_t ntiles64 = per_chunk * nzc * nrhs;
  if (ntiles64 > (1ll << 30)) return (int)hipErrorInvalidValue;
  const int ntiles = (int)ntiles64;
  dim3 blk(WV_LANES, 3), grd(w3_grid(ntiles, RG_ROWS * nfull + nrem));
  if (b)
    ELH_LAUNCH((k_apply3d_w3<T, TI, true>), grd, blk, 0, st, L, (const cx<TI>*)x, (const cx<T>*)b,
                       (cx<T>*)y, nfull, nrem, nzc, zc, ntiles);
  else
    ELH_LAUNCH((k_apply3d_w3<T, TI, false>), grd, blk, 0, st, L, (const cx<TI>*)x, (const cx<T>*)nullptr,
                       (cx<T>*)y, nfull, nrem, nzc, zc, ntiles);
  return (int)hipGetLastError();
}

template <typename T>
int launch_apply3d_w3_adj(const LevelArgs<T>& L, const void* x, const void* b, void* y, int nrhs, int zc,
                          hipStream_t st) {
  if (L.fs * (int64_t)sizeof(cx<T>) > (int64_t)0x7fffffff) return (int)hipErrorInvalidValue;
  int nfull = L.n[0] / WV_OUT, nrem = 0;  // as in launch_apply3d_w3
  const int rem = L.n[0] - nfull * WV_OUT;
  if (rem > RG_OUT) ++nfull;
  else if (rem > 0) nrem = 1;
  const int64_t per_chunk = (int64_t)(L.n[1] + RG_ROWS - 1) / RG_ROWS * (RG_ROWS * nfull + nrem);
  zc = w3_chunk(L.n, per_chunk, nrhs, zc);
  const int nzc = (L.n[2] + zc - 1) / zc;
  const int64_t ntiles64 = per_chunk * nzc * nrhs;
  if (ntiles64 > (1ll << 30)) return (int)hipErrorInvalidValue;
  const int ntiles = (int)ntiles64;
  dim3 blk(WV_LANES, 3), grd(w3_grid(ntiles, RG_ROWS * nfull + nrem));
  if (b)
    ELH_LAUNCH((k_apply3d_w3_adj<T, true>), grd, blk, 0, st, L, (const cx<T>*)x, (const cx<T>*)b,
                       (cx<T>*)y, nfull, nrem, nzc, zc, ntiles);
  else
    ELH_LAUNCH((k_apply3d_w3_adj<T, false>), grd, blk, 0, st, L, (const cx<T>*)x, (const cx<T>*)nullptr,
                       (cx<T>*)y, nfull, nrem, nzc, zc, ntiles);
  return (int)hipGetLastError();
}
template <typename T>
int launch_restrict_resid3d_w3(const LevelArgs<T>& F, const LevelArgs<T>& Cl, bool adj, const void* x,
                               const void* b, void* rc, int nrhs, int zc, hipStream_t st) {
  if (F.fs * (int64_t)sizeof(cx<T>) > (int64_t)0x7fffffff) return (int)hipErrorInvalidValue;
  if (!x || !b || (F.n[0] & 1) || (F.n[1] & 1) || (F.n[2] & 1) || Cl.n[0] * 2 != F.n[0] ||
      Cl.n[1] * 2 != F.n[1] || Cl.n[2] * 2 != F.n[2])
    return (int)hipErrorInvalidValue;
  const int tiles_x = (F.n[0] + (WV_OUT - 2) - 1) / (WV_OUT - 2);
  // chunk in coarse planes (same heuristic, counted on the coarse rows)
  const int nc[3] = {Cl.n[0], Cl.n[1], Cl.n[2]};
  zc = w3_chunk(nc, (int64_t)tiles_x * Cl.n[1], nrhs, zc);
  const int nzc = (Cl.n[2] + zc - 1) / zc;
  const int64_t ntiles64 = (int64_t)tiles_x * Cl.n[1] * nzc * nrhs;
  if (ntiles64 > (1ll << 30)) return (int)hipErrorInvalidValue;
  const int ntiles = (int)ntiles64;
  dim3 blk(WV_LANES, 7), grd(w3_grid(ntiles, 2 * tiles_x));
  if (adj)
    ELH_LAUNCH((k_restrict_resid3d_w3<T, true>), grd, blk, 0, st, F, Cl, (const cx<T>*)x, (const cx<T>*)b,
                       (cx<T>*)rc, tiles_x, nzc, zc, ntiles);
  else
    ELH_LAUNCH((k_restrict_resid3d_w3<T, false>), grd, blk, 0, st, F, Cl, (const cx<T>*)x,
                       (const cx<T>*)b, (cx<T>*)rc, tiles_x, nzc, zc, ntiles);
  return (int)hipGetLastError();
}
template int launch_restrict_resid3d_w3<double>(const LevelArgs<double>&, const LevelArgs<double>&, bool,
                                                const void*, const void*, void*, int, int, hipStream_t);
template int launch_restrict_resid3d_w3<float>(const LevelArgs<float>&, const LevelArgs<float>&, bool, const void*,
                                               const void*, void*, int, int, hipStream_t);

template int launch_apply3d_w3_adj<double>(const LevelArgs<double>&, const void*, const void*, void*, int, int,
                                           hipStream_t);
template int launch_apply3d_w3_adj<float>(const LevelArgs<float>&, const void*, const void*, void*, int, int,
                                          hipStream_t);

template int launch_apply3d_w3<double, double>(const LevelArgs<double>&, const void*, const void*, void*, int, int,
                                               hipStream_t);
template int launch_apply3d_w3<float, float>(const LevelArgs<float>&, const void*, const void*, void*, int, int,
                                             hipStream_t);
// float32 input, float64 arithmetic and output (the outer operator applied
// to float32 preconditioned vectors)
template int launch_apply3d_w3<double, float>(const LevelArgs<double>&, const void*, const void*, void*, int, int,
                                              hipStream_t);
}  // namespace elh
