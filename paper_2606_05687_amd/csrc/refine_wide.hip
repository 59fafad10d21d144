// FP64 refinement and certificate of problems with four contacts per stage
// (the feet and the hands of loco-manipulation, Sec. II-A: 24 inputs), one
// 64-lane wave per problem.
//
// The ADMM of Sec. III ends near the optimum; from its point the kernel runs a
// primal-dual interior point with Mehrotra's predictor-corrector on the QP
// (the same QP the two-contact refinement certifies), all in FP64:
//   rows     each stance contact's eleven wrench rows g_r . u_c <= h_r (Sec.
//            II-B, in the contact's own frame), scaled by m g (force rows) and
//            tau_max (moment rows), slacks s >= 0 and multipliers z >= 0;
//   Newton   every step is the LQ problem in (du, dx) with input Hessian
//            R' = R + G^T diag(z / s) G (per contact a 6 x 6 block; the
//            identity on a swing contact's inputs, which stay zero), linear
//            input term rho = R (u - u_ref) + G^T (z + (z rp - rc) / s) and
//            state term q = Q (x_{k+1} - r_k), solved by the backward Riccati
//            recursion over the horizon and a forward rollout of the gains;
//   stop     when the point's KKT residuals, with the interior point's own
//            multipliers, meet the tolerance.
// The returned u is the last iterate, x its rollout in FP64, and res its
// normalised residuals (r_dyn, r_ineq, r_stat, r_comp, r_sign).
//
// Per stage the wave forms, one entry per lane at a time through LDS, W B,
// W A and the system [H | Hwx | hw] with the input Hessian H = R' + B^T W B,
// Hwx = B^T W A and hw = rho + B^T w (W = S + Q, w = s + q, the value
// function (S, s) of x_{k+1}); lane c then holds column c of the system and
// one Gauss-Jordan elimination over the lanes (SPD, no pivoting) leaves the
// gains K = -H^{-1} Hwx and the feedforward kap = -H^{-1} hw in lanes
// 24..37; the value function of x_k is S = A^T W A + Hwx^T K,
// s = A^T w + Hwx^T kap (symmetrised).
#include "pinmpc_internal.h"

namespace pinmpc {

namespace {

constexpr int C4 = 4;                 // contacts
constexpr int U4 = 6 * C4;            // 24 inputs
constexpr int L4 = NX + U4;           // 37 lifted rows of the ADMM iterates
constexpr int TB = 36 + 6;            // per contact: R' block (6 x 6) and rho (6)
constexpr int NSN = NX * NX + NX;     // S and s of one stage

__device__ inline double wmax(double v) {
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
__device__ inline double wmin(double v) {
  for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
__device__ inline double wsum(double v) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// The kernel runs one 64-lane wave per workgroup.  LDS operations of a wave
// execute in issue order, so a hand-off between its lanes through LDS needs
// only a point the compiler moves no memory access across (wsync); the stage
// loops use it, so that loads of the next stage and stores of this one stay
// in flight across the hand-offs.  Data passed between lanes through global
// memory (one phase's results for the next) goes through the workgroup
// barrier with its memory fence at the phase boundaries.
__device__ inline void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Global pointers with their address space spelled out: the context is
// passed by reference into the phase functions, where a generic (flat)
// access would count against the LDS counter too, so that every wait for an
// LDS hand-off would also wait for the loads of the next stage in flight.
#define GMEM __attribute__((address_space(1)))
typedef const GMEM float* gcf;
typedef const GMEM double* gcd;
typedef GMEM double* gd;

// The problem's FP64 scratch (refine_wide_block_doubles(n) doubles).
struct WCtx {
  int b, n, N;
  double mu, fz, tm, mg, scf, scm;   // bounds, force scale, row scales
  gcf A, B, e, x_ref, u_ref, x0;
  const GMEM uint8_t* contact;       // [n][4]
  gd K, kap, u, du, x, dx, lam, T, s, z, ds, dz, rc, Hi, Hx;
};

static_assert(refine_wide_block_doubles(1) >=
                  (size_t)U4 * NX + 4 * U4 + C4 * TB + 5 * C4 * NROW + U4 * U4 + U4 * NX +
                      2 * 2 * NX,
              "the carve below fits the scratch block");

__device__ void carve(WCtx& C, gd blk) {
  const int n = C.n;
  C.K = blk;    blk += (size_t)n * U4 * NX;
  C.kap = blk;  blk += (size_t)n * U4;
  C.u = blk;    blk += (size_t)n * U4;
  C.du = blk;   blk += (size_t)n * U4;
  C.lam = blk;  blk += (size_t)n * U4;   // costates (13 used per stage)
  C.T = blk;    blk += (size_t)n * C4 * TB;
  C.s = blk;    blk += (size_t)n * C4 * NROW;
  C.z = blk;    blk += (size_t)n * C4 * NROW;
  C.ds = blk;   blk += (size_t)n * C4 * NROW;
  C.dz = blk;   blk += (size_t)n * C4 * NROW;
  C.rc = blk;   blk += (size_t)n * C4 * NROW;
  C.Hi = blk;   blk += (size_t)n * U4 * U4;
  C.Hx = blk;   blk += (size_t)n * U4 * NX;
  C.x = blk;    blk += (size_t)(n + 1) * NX;
  C.dx = blk;
}

// LDS of the stage recursion.
// Matrices with 13 columns keep rows of 14 (XP), so that an entry with an even
// column and its right neighbour are one aligned 16-byte pair; the stage
// products read such pairs.
constexpr int XP = NX + 1;
// Arrays whose lives within a stage do not overlap share storage, which keeps
// a workgroup within 20 KB of LDS (eight per compute unit):
//   X: B, W B and the stage terms, from the stage's start to the system;
//   Y: the system [H | Hwx | hw] column by column until the elimination reads
//      it; then the gains by column with the feedforward, and the unsymmetrised
//      value function, over the H columns, while the Hwx columns stay for the
//      value-function update.
constexpr int OFF_WB = NX * U4, OFF_T = 2 * NX * U4;        // in X
constexpr int OFF_HWX = U4 * U4, OFF_SN = (NX + 1) * U4;     // in Y
static_assert(OFF_SN + NSN <= OFF_HWX, "gains and value function fit over the H columns");
struct WSh {
  alignas(16) double A[NX * XP];
  alignas(16) double WA[NX * XP];
  alignas(16) double X[2 * NX * U4 + C4 * TB];
  alignas(16) double Y[(L4 + 1) * U4];
  double W[NX * NX];   // S + Q of x_{k+1}, formed when S is
  double sv[NX], w[NX], kap[U4], v13[NX], v24[U4], Q[NX], R[U4];
};

typedef double dpair __attribute__((ext_vector_type(2)));
__device__ inline dpair ld2(const double* p) { return *reinterpret_cast<const dpair*>(p); }
__device__ inline void st2(double* p, double a, double b) {
  *reinterpret_cast<dpair*>(p) = dpair{a, b};
}
__device__ inline void st2(gd p, double a, double b) {
  *reinterpret_cast<GMEM dpair*>(p) = dpair{a, b};
}

__device__ inline bool stance(const WCtx& C, int k, int i) { return C.contact[k * C4 + i] != 0; }

// g_r . u for the eleven rows of one contact (u its six inputs), with h_r and
// the row scale: pyramid sides, normal-force bound, moment box.
__device__ inline void rows_of(const WCtx& C, const double u[6], double gu[NROW], double h[NROW],
                               double sc[NROW]) {
  gu[0] = u[0] - C.mu * u[2];
  gu[1] = -u[0] - C.mu * u[2];
  gu[2] = u[1] - C.mu * u[2];
  gu[3] = -u[1] - C.mu * u[2];
  gu[4] = u[2];
  #pragma unroll
  for (int a = 0; a < 3; ++a) {
    gu[5 + a] = u[3 + a];
    gu[8 + a] = -u[3 + a];
  }
  #pragma unroll
  for (int r = 0; r < NROW; ++r) {
    h[r] = r < 4 ? 0.0 : (r == 4 ? C.fz : C.tm);
    sc[r] = r < 5 ? C.scf : C.scm;
  }
}

// G^T v for one contact (v one value per row).
__device__ inline void rows_T(const WCtx& C, const double v[NROW], double o[6]) {
  o[0] = v[0] - v[1];
  o[1] = v[2] - v[3];
  o[2] = -C.mu * (v[0] + v[1] + v[2] + v[3]) + v[4];
  #pragma unroll
  for (int a = 0; a < 3; ++a) o[3 + a] = v[5 + a] - v[8 + a];
}

__device__ inline void ld6(gcd p, double v[6]) {
  #pragma unroll
  for (int t = 0; t < 6; ++t) v[t] = p[t];
}
__device__ inline void ldr(gcd p, double v[NROW]) {
  #pragma unroll
  for (int r = 0; r < NROW; ++r) v[r] = p[r];
}
__device__ inline void str(gd p, const double v[NROW]) {
  #pragma unroll
  for (int r = 0; r < NROW; ++r) p[r] = v[r];
}

// Stage input terms of the Newton step, in parallel over (stage, contact):
// the R' block and rho of every contact (identity and zero on a swing
// contact), from the iterate (u, s, z) and the complementarity target rc.
template <int OCC>
__device__ __attribute__((noinline)) void build_terms(const WCtx& C, const WSh& sh) {
  __syncthreads();
  for (int e = threadIdx.x; e < C.N * C4; e += 64) {
    const int k = e / C4, i = e % C4;
    gd T = C.T + (size_t)e * TB;
    if (!stance(C, k, i)) {
      #pragma unroll
      for (int t = 0; t < 36; ++t) T[t] = (t % 7 == 0) ? 1.0 : 0.0;
      #pragma unroll
      for (int t = 0; t < 6; ++t) T[36 + t] = 0.0;
      continue;
    }
    double u[6], gu[NROW], h[NROW], sc[NROW], sv[NROW], zv[NROW], cv[NROW];
    ld6(C.u + (size_t)k * U4 + 6 * i, u);
    ldr(C.s + (size_t)e * NROW, sv);
    ldr(C.z + (size_t)e * NROW, zv);
    ldr(C.rc + (size_t)e * NROW, cv);
    rows_of(C, u, gu, h, sc);
    double d[NROW], c[NROW];
    #pragma unroll
    for (int r = 0; r < NROW; ++r) {
      const double rp = (gu[r] - h[r]) / sc[r] + sv[r];
      d[r] = zv[r] / (sv[r] * sc[r] * sc[r]);
      c[r] = (zv[r] + (zv[r] * rp - cv[r]) / sv[r]) / sc[r];
    }
    double H[36];
    #pragma unroll
    for (int t = 0; t < 36; ++t) H[t] = 0.0;
    const double m = C.mu;
    H[0 * 6 + 0] = d[0] + d[1];
    H[0 * 6 + 2] = H[2 * 6 + 0] = -m * (d[0] - d[1]);
    H[1 * 6 + 1] = d[2] + d[3];
    H[1 * 6 + 2] = H[2 * 6 + 1] = -m * (d[2] - d[3]);
    H[2 * 6 + 2] = m * m * (d[0] + d[1] + d[2] + d[3]) + d[4];
    #pragma unroll
    for (int a = 0; a < 3; ++a) H[(3 + a) * 7] = d[5 + a] + d[8 + a];
    double rho[6];
    rows_T(C, c, rho);
    #pragma unroll
    for (int t = 0; t < 6; ++t) {
      const int j = 6 * i + t;
      const double ur = C.u_ref ? (double)C.u_ref[(size_t)k * U4 + j] : 0.0;
      H[t * 7] += sh.R[j];
      rho[t] += sh.R[j] * (u[t] - ur);
    }
    #pragma unroll
    for (int t = 0; t < 36; ++t) T[t] = H[t];
    #pragma unroll
    for (int t = 0; t < 6; ++t) T[36 + t] = rho[t];
  }
  __syncthreads();
}

// Backward recursion of the Newton step, stages N-1 .. 0: gains and
// feedforward of every stage into the scratch.  The elimination also turns the
// identity carried in lanes 38..61 into H^{-1}, kept with Hwx for a second
// right-hand side of the same Newton matrix (factor = false: the corrector of
// an interior-point iteration), whose recursion is the vector part alone:
// hw = rho + B^T w, kap = -H^{-1} hw, s = A^T w + Hwx^T kap.
template <int OCC>
__device__ __attribute__((noinline)) void backward_rhs(const WCtx& C, WSh& sh) {
  const int lane = threadIdx.x;
  __syncthreads();
  {
    if (lane < NX) sh.sv[lane] = 0.0;
    // per stage: lanes 0..23 the linear term and their column of B, lanes
    // 0..12 x_{k+1}, x_ref[k] and their column of A, fetched a stage ahead
    // from clamped addresses; the rows of H^{-1} and columns of Hwx at the
    // top of their own stage
    const int lu = min(lane, U4 - 1), lx = min(lane, NX - 1);
    double frho, fx, fr;
    float fbc[NX], fac[NX];
    auto fetch = [&](int k) {
      frho = C.T[(size_t)k * C4 * TB + (lu / 6) * TB + 36 + lu % 6];
      const auto Bk = C.B + (size_t)k * NX * U4;
      const auto Ak = C.A + (size_t)k * NX * NX;
#pragma unroll
      for (int i = 0; i < NX; ++i) {
        fbc[i] = Bk[i * U4 + lu];
        fac[i] = Ak[i * NX + lx];
      }
      fx = C.x[(size_t)(k + 1) * NX + lx];
      fr = (double)C.x_ref[(size_t)k * NX + lx];
    };
    fetch(C.N - 1);
    for (int k = C.N - 1; k >= 0; --k) {
      double h[U4], hw[U4], rho = frho, bc[NX], ac[NX];
      const auto Hc = C.Hi + (size_t)k * U4 * U4 + lu;
      const auto Hx = C.Hx + (size_t)k * U4 * NX + lx;
#pragma unroll
      for (int j = 0; j < U4; ++j) {
        h[j] = Hc[j * U4];
        hw[j] = Hx[j * NX];
      }
#pragma unroll
      for (int i = 0; i < NX; ++i) {
        bc[i] = (double)fbc[i];
        ac[i] = (double)fac[i];
      }
      const double q = sh.Q[lx] * (fx - fr);
      fetch(k > 0 ? k - 1 : 0);   // in flight during this stage
      wsync();
      if (lane < NX) sh.w[lane] = sh.sv[lane] + q;
      wsync();
      if (lane < U4) {
        // swing inputs: zero rho and a unit row of H^{-1}, so kap = 0 there
        double a = rho;
        if (stance(C, k, lane / 6)) {
#pragma unroll
          for (int i = 0; i < NX; ++i) a = fma(bc[i], sh.w[i], a);
        }
        sh.v24[lane] = a;
      }
      wsync();
      if (lane < U4) {
        // row `lane` of H^{-1} (its columns are stored one after the other)
        double a = 0.0;
#pragma unroll
        for (int j = 0; j < U4; ++j) a = fma(h[j], sh.v24[j], a);
        sh.kap[lane] = -a;
        C.kap[(size_t)k * U4 + lane] = -a;
      }
      if (k == 0) break;
      wsync();
      if (lane < NX) {
        double a = 0.0;
#pragma unroll
        for (int l = 0; l < NX; ++l) a = fma(ac[l], sh.w[l], a);
#pragma unroll
        for (int r = 0; r < U4; ++r) a = fma(hw[r], sh.kap[r], a);
        sh.sv[lane] = a;
      }
    }
    __syncthreads();
  }
}

template <int OCC>
__device__ __attribute__((noinline)) void backward(const WCtx& C, WSh& sh, bool factor) {
  if (!factor) {
    backward_rhs<OCC>(C, sh);
    return;
  }
  const int lane = threadIdx.x;
  double* const B = sh.X;
  double* const WB = sh.X + OFF_WB;
  double* const T = sh.X + OFF_T;
  double* const Aug = sh.Y;
  double* const Kc = sh.Y;
  double* const Sn = sh.Y + OFF_SN;
  __syncthreads();
  for (int e = lane; e < NX * NX; e += 64) sh.W[e] = (e % (NX + 1) == 0) ? sh.Q[e / NX] : 0.0;
  if (lane < NX) sh.sv[lane] = 0.0;
  // the stage data a lane moves into LDS (A: 3, B: 5, stage terms: 3 items per
  // lane; x_{k+1} and x_ref[k] in lanes 0..12; the contact flags), fetched a
  // stage ahead; the addresses are clamped into the stage's arrays, so every
  // lane issues the same loads on every path
  float fa[3], fb[5];
  double ft[3], fx, fr;
  uint32_t fc;
  auto fetch = [&](int k) {
    fc = *reinterpret_cast<const GMEM uint32_t*>(C.contact + (size_t)k * C4);
    const auto Ak = C.A + (size_t)k * NX * NX;
    const auto Bk = C.B + (size_t)k * NX * U4;
    const auto Tk = C.T + (size_t)k * C4 * TB;
#pragma unroll
    for (int i = 0; i < 3; ++i) fa[i] = Ak[min(lane + 64 * i, NX * NX - 1)];
#pragma unroll
    for (int i = 0; i < 5; ++i) fb[i] = Bk[min(lane + 64 * i, NX * U4 - 1)];
#pragma unroll
    for (int i = 0; i < 3; ++i) ft[i] = Tk[min(lane + 64 * i, C4 * TB - 1)];
    const int l = min(lane, NX - 1);
    fx = C.x[(size_t)(k + 1) * NX + l];
    fr = (double)C.x_ref[(size_t)k * NX + l];
  };
  fetch(C.N - 1);
  for (int k = C.N - 1; k >= 0; --k) {
    // with two waves per SIMD the lane index is opaque to the compiler once
    // per stage: the per-lane LDS addresses below are then formed anew each
    // stage (a few integer operations) instead of held in registers across
    // it, which lets the two waves share a SIMD without spilling inside it
    int lane_k = threadIdx.x;
    if constexpr (OCC > 1) asm volatile("" : "+v"(lane_k));
    const int lane = lane_k;
    wsync();
    uint32_t unit = 0;
    #pragma unroll
    for (int i = 0; i < C4; ++i)
      if (((fc >> (8 * i)) & 0xFFu) == 0) unit |= 0x3Fu << (6 * i);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int e = lane + 64 * i;
      if (e < NX * NX) sh.A[(e / NX) * XP + e % NX] = (double)fa[i];
      if (e < C4 * TB) T[e] = ft[i];
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      const int e = lane + 64 * i;
      if (e < NX * U4) B[e] = ((unit >> (e % U4)) & 1u) ? 0.0 : (double)fb[i];
    }
    if (lane < NX) sh.w[lane] = sh.sv[lane] + sh.Q[lane] * (fx - fr);
    fetch(k > 0 ? k - 1 : 0);   // in flight during this stage
    wsync();
    // W B and W A in blocks of two neighbouring entries of a row (each entry
    // summed in the order of its own dot product)
    for (int e = lane; e < NX * (U4 / 2) + NX * 7; e += 64) {
      double a0 = 0.0, a1 = 0.0;
      if (e < NX * (U4 / 2)) {
        const int i = e / (U4 / 2), c = 2 * (e % (U4 / 2));
#pragma unroll
        for (int j = 0; j < NX; ++j) {
          const double w = sh.W[i * NX + j];
          const dpair b = ld2(&B[j * U4 + c]);
          a0 = fma(w, b.x, a0);
          a1 = fma(w, b.y, a1);
        }
        st2(&WB[i * U4 + c], a0, a1);
      } else {
        const int f = e - NX * (U4 / 2), i = f / 7, j = 2 * (f % 7);
#pragma unroll
        for (int l = 0; l < NX; ++l) {
          const double w = sh.W[i * NX + l];
          const dpair b = ld2(&sh.A[l * XP + j]);
          a0 = fma(w, b.x, a0);
          a1 = fma(w, b.y, a1);
        }
        st2(&sh.WA[i * XP + j], a0, a1);   // column 13 of the pair is padding
      }
    }
    wsync();
    // the columns of [H | Hwx | hw] (column c at Aug[c][0..23]) in blocks of
    // two rows r, r + 1: H = R' + B^T (W B) two columns at a time,
    // Hwx = B^T (W A) and hw = rho + B^T w one column at a time
    for (int e = lane; e < 12 * 12 + 12 * NX + 12; e += 64) {
      if (e < 144) {
        const int r = 2 * (e / 12), c = 2 * (e % 12);
        double a00, a01, a10, a11;   // (r, c), (r, c+1), (r+1, c), (r+1, c+1)
        if (r / 6 == c / 6) {
          const double* Tb = T + (c / 6) * TB;
          const int rr = r % 6, cc = c % 6;
          a00 = Tb[rr * 6 + cc];
          a01 = Tb[rr * 6 + cc + 1];
          a10 = Tb[(rr + 1) * 6 + cc];
          a11 = Tb[(rr + 1) * 6 + cc + 1];
        } else {
          a00 = a01 = a10 = a11 = 0.0;
        }
#pragma unroll
        for (int i = 0; i < NX; ++i) {
          const dpair b = ld2(&B[i * U4 + r]);
          const dpair g = ld2(&WB[i * U4 + c]);
          a00 = fma(b.x, g.x, a00);
          a01 = fma(b.x, g.y, a01);
          a10 = fma(b.y, g.x, a10);
          a11 = fma(b.y, g.y, a11);
        }
        st2(&Aug[c * U4 + r], a00, a10);
        st2(&Aug[(c + 1) * U4 + r], a01, a11);
      } else if (e < 144 + 12 * NX) {
        const int f = e - 144, r = 2 * (f / NX), j = f % NX;
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int i = 0; i < NX; ++i) {
          const dpair b = ld2(&B[i * U4 + r]);
          const double g = sh.WA[i * XP + j];
          a0 = fma(b.x, g, a0);
          a1 = fma(b.y, g, a1);
        }
        C.Hx[(size_t)k * U4 * NX + r * NX + j] = a0;
        C.Hx[(size_t)k * U4 * NX + (r + 1) * NX + j] = a1;
        st2(&Aug[(U4 + j) * U4 + r], a0, a1);
      } else {
        const int r = 2 * (e - 144 - 12 * NX);
        double a0 = T[(r / 6) * TB + 36 + r % 6];
        double a1 = T[((r + 1) / 6) * TB + 36 + (r + 1) % 6];
#pragma unroll
        for (int i = 0; i < NX; ++i) {
          const dpair b = ld2(&B[i * U4 + r]);
          const double g = sh.w[i];
          a0 = fma(b.x, g, a0);
          a1 = fma(b.y, g, a1);
        }
        st2(&Aug[L4 * U4 + r], a0, a1);
      }
    }
    wsync();
    double col[U4];
#pragma unroll
    for (int r = 0; r < U4; ++r)
      col[r] = lane <= L4 ? Aug[lane * U4 + r] : (lane - L4 - 1 == r ? 1.0 : 0.0);
    gj_columns<U4>(col, unit);
    // lanes 24..36: the gain columns -H^{-1} Hwx; lane 37: the feedforward
    // -H^{-1} hw; lanes 38..61: the columns of H^{-1}; each a contiguous
    // column of 24 in the scratch (and the gains with the feedforward in LDS)
    if (lane >= U4 && lane < L4 + 1 + U4) {
      const double sg = lane <= L4 ? -1.0 : 1.0;
      gd dst = lane < L4 ? C.K + (size_t)k * U4 * NX + (lane - U4) * U4
                  : lane == L4 ? C.kap + (size_t)k * U4
                               : C.Hi + (size_t)k * U4 * U4 + (lane - L4 - 1) * U4;
#pragma unroll
      for (int r = 0; r < U4; r += 2) st2(dst + r, sg * col[r], sg * col[r + 1]);
      if (lane <= L4) {
#pragma unroll
        for (int r = 0; r < U4; r += 2) st2(&Kc[(lane - U4) * U4 + r], -col[r], -col[r + 1]);
      }
    }
    if (k == 0) break;   // x_0 is fixed: its value function is not needed
    wsync();
    // S = A^T W A + Hwx^T K and s = A^T w + Hwx^T kap in blocks of two rows
    // i, i + 1 (row 13 of the last block is padding)
    for (int e = lane; e < 7 * (NX + 1); e += 64) {
      const int i = 2 * (e / (NX + 1)), j = e % (NX + 1);   // j = 13: s
      double a0 = 0.0, a1 = 0.0;
#pragma unroll
      for (int l = 0; l < NX; ++l) {
        const dpair av = ld2(&sh.A[l * XP + i]);
        const double g = j < NX ? sh.WA[l * XP + j] : sh.w[l];
        a0 = fma(av.x, g, a0);
        a1 = fma(av.y, g, a1);
      }
#pragma unroll
      for (int r = 0; r < U4; ++r) {
        // Hwx (r, i) and (r, i + 1): rows r of the system's columns 24 + i, 25 + i
        const double h0 = Aug[OFF_HWX + i * U4 + r];
        const double h1 = i + 1 < NX ? Aug[OFF_HWX + (i + 1) * U4 + r] : 0.0;
        const double g = Kc[j * U4 + r];
        a0 = fma(h0, g, a0);
        a1 = fma(h1, g, a1);
      }
      if (j < NX) {
        Sn[i * NX + j] = a0;
        if (i + 1 < NX) Sn[(i + 1) * NX + j] = a1;
      } else {
        Sn[NX * NX + i] = a0;
        if (i + 1 < NX) Sn[NX * NX + i + 1] = a1;
      }
    }
    wsync();
    for (int e = lane; e < NX * NX; e += 64) {
      const int i = e / NX, j = e % NX;
      const double s = 0.5 * (Sn[i * NX + j] + Sn[j * NX + i]);
      sh.W[e] = s + (i == j ? sh.Q[i] : 0.0);
    }
    if (lane < NX) sh.sv[lane] = Sn[NX * NX + lane];
  }
  __syncthreads();
}

// Forward rollout of the gains from dx_0 = 0: du_k = K_k dx_k + kap_k,
// dx_{k+1} = A_k dx_k + B_k du_k.
template <int OCC>
__device__ __attribute__((noinline)) void forward(const WCtx& C, WSh& sh) {
  const int lane = threadIdx.x;
  __syncthreads();
  if (lane < NX) {
    sh.v13[lane] = 0.0;
    C.dx[lane] = 0.0;
  }
  // a stage's gains row and feedforward (lanes 0..23) and rows of A and B
  // (lanes 0..12), fetched a stage ahead from clamped addresses
  const int lk = min(lane, U4 - 1), lx = min(lane, NX - 1);
  double fk[NX], fp;
  float fa[NX], fb[U4];
  auto fetch = [&](int k) {
    const auto Kr = C.K + (size_t)k * U4 * NX + lk;   // row lk of K (stored by column)
#pragma unroll
    for (int c = 0; c < NX; ++c) fk[c] = Kr[c * U4];
    fp = C.kap[(size_t)k * U4 + lk];
    const auto Ar = C.A + (size_t)k * NX * NX + lx * NX;
    const auto Br = C.B + (size_t)k * NX * U4 + lx * U4;
#pragma unroll
    for (int c = 0; c < NX; ++c) fa[c] = Ar[c];
#pragma unroll
    for (int r = 0; r < U4; ++r) fb[r] = Br[r];
  };
  fetch(0);
  for (int k = 0; k < C.N; ++k) {
    double kr[NX], kp = fp;
    float ar[NX], br[U4];
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      kr[c] = fk[c];
      ar[c] = fa[c];
    }
#pragma unroll
    for (int r = 0; r < U4; ++r) br[r] = fb[r];
    fetch(k + 1 < C.N ? k + 1 : k);   // in flight during this stage
    wsync();
    if (lane < U4) {
      double a = kp;
      #pragma unroll
      for (int c = 0; c < NX; ++c) a = fma(kr[c], sh.v13[c], a);
      sh.v24[lane] = a;
      C.du[(size_t)k * U4 + lane] = a;
    }
    wsync();
    double nx = 0.0;
    if (lane < NX) {
      #pragma unroll
      for (int c = 0; c < NX; ++c) nx = fma((double)ar[c], sh.v13[c], nx);
      #pragma unroll
      for (int r = 0; r < U4; ++r) nx = fma((double)br[r], sh.v24[r], nx);
      C.dx[(size_t)(k + 1) * NX + lane] = nx;
    }
    wsync();
    if (lane < NX) sh.v13[lane] = nx;
  }
  __syncthreads();
}

// FP64 rollout of u from x0 into x, and the dynamics residual of that
// trajectory (normalised as the certificate's r_dyn).
template <int OCC>
__device__ __attribute__((noinline)) double rollout(const WCtx& C, WSh& sh) {
  const int lane = threadIdx.x;
  __syncthreads();
  if (lane < NX) {
    const double v = (double)C.x0[lane];
    sh.v13[lane] = v;
    C.x[lane] = v;
  }
  double rd = 0.0;
  for (int k = 0; k < C.N; ++k) {
    __syncthreads();
    double nx = 0.0, ax = 0.0, bu = 0.0;
    if (lane < NX) {
      const auto Ar = C.A + (size_t)k * NX * NX + lane * NX;
      const auto Br = C.B + (size_t)k * NX * U4 + lane * U4;
      const auto uk = C.u + (size_t)k * U4;
      #pragma unroll
      for (int c = 0; c < NX; ++c) ax = fma((double)Ar[c], sh.v13[c], ax);
      #pragma unroll
      for (int r = 0; r < U4; ++r) bu = fma((double)Br[r], uk[r], bu);
      const double ev = C.e ? (double)C.e[(size_t)k * NX + lane] : 0.0;
      nx = ax + bu + ev;
      C.x[(size_t)(k + 1) * NX + lane] = nx;
    }
    // |x_{k+1} - A x_k - B u_k - e_k| over the stage's largest term
    const double d = fabs(nx - ax - bu - (lane < NX && C.e ? (double)C.e[(size_t)k * NX + lane] : 0.0));
    const double den = 1.0 + wmax(fmax(fabs(nx), fmax(fabs(ax), fabs(bu))));
    rd = fmax(rd, wmax(d) / den);
    __syncthreads();
    if (lane < NX) sh.v13[lane] = nx;
  }
  __syncthreads();
  return rd;
}

// Gradient of force row r (0..4) of the pyramid with respect to f.
__device__ inline void frow(int r, double mu, double g[3]) {
  g[0] = r == 0 ? 1.0 : (r == 1 ? -1.0 : 0.0);
  g[1] = r == 2 ? 1.0 : (r == 3 ? -1.0 : 0.0);
  g[2] = r == 4 ? 1.0 : -mu;
}

// Multipliers m >= 0 of the force rows in the set `am` (bits 0..4) that best
// cancel the force gradient gf: min |gf + sum_r m_r g_r| (nonnegative least
// squares).  An optimal support has at most three independent rows, so the
// candidates are every subset of at most three rows of `am` with a
// nonsingular Gram matrix whose least-squares multipliers are nonnegative.
// Every loop below unrolls completely (the subset S is a constant in each
// copy), so no array is indexed at run time and all of them stay in registers.
__device__ void force_refit(int am, double mu, const double gf[3], double m[5]) {
  double best = gf[0] * gf[0] + gf[1] * gf[1] + gf[2] * gf[2];
#pragma unroll
  for (int t = 0; t < 5; ++t) m[t] = 0.0;
  const double scale = 1.0 + mu * mu;
#pragma unroll
  for (int S = 1; S < 32; ++S) {
    if (__builtin_popcount(S) > 3) continue;
    if ((S & am) != S) continue;
    int idx[3] = {0, 0, 0}, k = 0;
#pragma unroll
    for (int r = 0; r < 5; ++r)
      if ((S >> r) & 1) idx[k++] = r;
    double g[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j) frow(j < k ? idx[j] : 0, mu, g[j]);
    // Gram matrix and right-hand side -G_S gf (k x k, k <= 3), the identity
    // on the unused rows
    double M[3][3], b[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      b[a] = a < k ? -(g[a][0] * gf[0] + g[a][1] * gf[1] + g[a][2] * gf[2]) : 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c)
        M[a][c] = (a < k && c < k) ? g[a][0] * g[c][0] + g[a][1] * g[c][1] + g[a][2] * g[c][2]
                                   : (a == c ? 1.0 : 0.0);
    }
    const double det = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
                       M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                       M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
    if (!(fabs(det) > 1e-10 * scale * scale * scale)) continue;   // dependent rows
    double x[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double D[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) D[i][c] = c == a ? b[i] : M[i][c];
      x[a] = (D[0][0] * (D[1][1] * D[2][2] - D[1][2] * D[2][1]) -
              D[0][1] * (D[1][0] * D[2][2] - D[1][2] * D[2][0]) +
              D[0][2] * (D[1][0] * D[2][1] - D[1][1] * D[2][0])) / det;
    }
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) ok = ok && (a >= k || x[a] >= 0.0);
    if (!ok) continue;
    double rv[3] = {gf[0], gf[1], gf[2]};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) rv[c] += a < k ? x[a] * g[a][c] : 0.0;
    const double res = rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2];
    if (res < best) {
      best = res;
#pragma unroll
      for (int t = 0; t < 5; ++t) {
        double v = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) v = (a < k && idx[a] == t) ? x[a] : v;
        m[t] = v;
      }
    }
  }
}

// The certificate of the iterate: x (rollout of u) and res.  The costates
// come from the adjoint recursion; each stance contact's row multipliers are
// refitted to its input gradient on the rows whose slack is at most tol times
// the row's scale (nonnegative least squares: the force rows by force_refit,
// each moment axis in closed form), so complementarity holds to tol by
// construction and stationarity measures how well u meets it.  (The interior
// point's own multipliers lose their accuracy as the slacks of active rows
// approach zero: their step divides by the slack.)  Returns max(res).
template <int OCC>
__device__ __attribute__((noinline)) double certificate(const WCtx& C, WSh& sh, double res[PINMPC_NRES],
                                                      double tol) {
  const int lane = threadIdx.x;
  res[0] = rollout<OCC>(C, sh);
  // costates, backwards: lam_k = Q (x_{k+1} - r_k) + A_{k+1}^T lam_{k+1}
  double tq = 0.0, tl = 0.0, ta = 0.0;
  if (lane < NX) sh.v13[lane] = 0.0;
  for (int k = C.N - 1; k >= 0; --k) {
    __syncthreads();
    double l = 0.0, al = 0.0;
    if (lane < NX) {
      const double q =
          sh.Q[lane] * (C.x[(size_t)(k + 1) * NX + lane] - (double)C.x_ref[(size_t)k * NX + lane]);
      if (k + 1 < C.N) {
        const auto A1 = C.A + (size_t)(k + 1) * NX * NX;
        #pragma unroll
        for (int i = 0; i < NX; ++i) al = fma((double)A1[i * NX + lane], sh.v13[i], al);
      }
      l = q + al;
      C.lam[(size_t)k * U4 + lane] = l;
      tq = fmax(tq, fabs(q));
      tl = fmax(tl, fabs(l));
      ta = fmax(ta, fabs(al));
    }
    __syncthreads();
    if (lane < NX) sh.v13[lane] = l;
  }
  __syncthreads();
  // per (stage, contact): gradient, multipliers, feasibility, complementarity
  double terms = fmax(tq, fmax(tl, ta)), stat = 0.0, rin = 0.0, mmax = 0.0, comp = 0.0;
  for (int e = lane; e < C.N * C4; e += 64) {
    const int k = e / C4, i = e % C4;
    double u[6];
    ld6(C.u + (size_t)k * U4 + 6 * i, u);
    if (!stance(C, k, i)) {
      #pragma unroll
      for (int t = 0; t < 6; ++t) rin = fmax(rin, fabs(u[t]) / C.mg);
      continue;
    }
    double gu[NROW], h[NROW], sc[NROW], mv[NROW], gr[6];
    rows_of(C, u, gu, h, sc);
    const auto Bk = C.B + (size_t)k * NX * U4;
    const auto lk = C.lam + (size_t)k * U4;
    double tr = 0.0, tb = 0.0;
#pragma unroll
    for (int t = 0; t < 6; ++t) {
      const int j = 6 * i + t;
      const double ur = C.u_ref ? (double)C.u_ref[(size_t)k * U4 + j] : 0.0;
      const double ru = sh.R[j] * (u[t] - ur);
      double bl = 0.0;
#pragma unroll
      for (int l = 0; l < NX; ++l) bl = fma((double)Bk[l * U4 + j], lk[l], bl);
      tr = fmax(tr, fabs(ru));
      tb = fmax(tb, fabs(bl));
      gr[t] = ru + bl;
    }
    // rows active within tol, their refitted multipliers
    int am = 0;
#pragma unroll
    for (int r = 0; r < NROW; ++r)
      if (h[r] - gu[r] <= tol * sc[r]) am |= 1 << r;
    double mf[5];
    force_refit(am & 31, C.mu, gr, mf);
#pragma unroll
    for (int r = 0; r < 5; ++r) mv[r] = mf[r];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      mv[5 + a] = ((am >> (5 + a)) & 1) ? fmax(-gr[3 + a], 0.0) : 0.0;
      mv[8 + a] = ((am >> (8 + a)) & 1) ? fmax(gr[3 + a], 0.0) : 0.0;
    }
    double gm[6];
    rows_T(C, mv, gm);
    double tg = 0.0, cmp = 0.0;
#pragma unroll
    for (int t = 0; t < 6; ++t) {
      tg = fmax(tg, fabs(gm[t]));
      stat = fmax(stat, fabs(gr[t] + gm[t]));
    }
#pragma unroll
    for (int r = 0; r < NROW; ++r) {
      rin = fmax(rin, fmax(gu[r] - h[r], 0.0) / C.mg);
      mmax = fmax(mmax, mv[r]);
      cmp = fmax(cmp, mv[r] * fmax(h[r] - gu[r], 0.0));
    }
    comp = fmax(comp, cmp);
    terms = fmax(terms, fmax(tr, fmax(tb, tg)));
  }
  terms = wmax(terms);
  mmax = wmax(mmax);
  comp = wmax(comp) / (1.0 + mmax * C.mg);
  res[1] = wmax(rin);
  res[2] = wmax(stat) / (1.0 + terms);
  res[3] = comp;
  res[4] = 0.0;   // the refitted multipliers are nonnegative
  double m = 0.0;
  #pragma unroll
  for (int i = 0; i < PINMPC_NRES; ++i) m = fmax(m, res[i]);
  return m;
}

// Slack and multiplier steps of the direction (du) for complementarity
// target rc; returns the largest step keeping s, z >= 0 (at most 1).
template <int OCC>
__device__ __attribute__((noinline)) double row_steps(const WCtx& C) {
  double amax = 1.0;
  for (int e = threadIdx.x; e < C.N * C4; e += 64) {
    const int k = e / C4, i = e % C4;
    if (!stance(C, k, i)) continue;
    double u[6], du[6], gu[NROW], gd[NROW], h[NROW], sc[NROW], sv[NROW], zv[NROW], cv[NROW];
    ld6(C.u + (size_t)k * U4 + 6 * i, u);
    ld6(C.du + (size_t)k * U4 + 6 * i, du);
    ldr(C.s + (size_t)e * NROW, sv);
    ldr(C.z + (size_t)e * NROW, zv);
    ldr(C.rc + (size_t)e * NROW, cv);
    rows_of(C, u, gu, h, sc);
    rows_of(C, du, gd, h, sc);
    double dsv[NROW], dzv[NROW];
    #pragma unroll
    for (int r = 0; r < NROW; ++r) {
      const double rp = (gu[r] - h[r]) / sc[r] + sv[r];
      dsv[r] = -rp - gd[r] / sc[r];
      dzv[r] = (-cv[r] - zv[r] * dsv[r]) / sv[r];
      if (dsv[r] < 0.0) amax = fmin(amax, -sv[r] / dsv[r]);
      if (dzv[r] < 0.0) amax = fmin(amax, -zv[r] / dzv[r]);
    }
    str(C.ds + (size_t)e * NROW, dsv);
    str(C.dz + (size_t)e * NROW, dzv);
  }
  return wmin(amax);
}

// Interior point from the current u (its rollout in x).  Returns the
// iterations; *ok tells whether the certificate was met (then res is it).
template <int OCC>
__device__ __attribute__((noinline)) int ipm(const WCtx& C, WSh& sh, int maxit, double tol, double res[PINMPC_NRES],
                   bool* ok, int* nfact) {
  const int lane = threadIdx.x;
  *ok = false;
  *nfact = 0;   // backward recursions that factored (the others: vector part only)
  // rows of stance contacts, starting slacks (at least 1) and multipliers 1
  double mloc = 0.0, smz = 0.0, rpn = 0.0;
  __syncthreads();
  for (int e = lane; e < C.N * C4; e += 64) {
    const int k = e / C4, i = e % C4;
    if (!stance(C, k, i)) continue;
    double u[6], gu[NROW], h[NROW], sc[NROW], sv[NROW], zv[NROW];
    ld6(C.u + (size_t)k * U4 + 6 * i, u);
    rows_of(C, u, gu, h, sc);
    #pragma unroll
    for (int r = 0; r < NROW; ++r) {
      sv[r] = fmax((h[r] - gu[r]) / sc[r], 1.0);
      zv[r] = 1.0;
      smz += sv[r] * zv[r];
      rpn = fmax(rpn, fabs((gu[r] - h[r]) / sc[r] + sv[r]));
    }
    mloc += NROW;
    str(C.s + (size_t)e * NROW, sv);
    str(C.z + (size_t)e * NROW, zv);
    str(C.rc + (size_t)e * NROW, sv);   // affine target s z with z = 1
  }
  const double m = wsum(mloc);
  int it = 0;
  for (; it < maxit; ++it) {
    const double muv = m > 0.0 ? wsum(smz) / m : 0.0;
    rpn = wmax(rpn);
    if (muv <= 1e-8 && rpn <= 1e-8) {
      if (certificate<OCC>(C, sh, res, tol) <= tol) {
        *ok = true;
        return it;
      }
      // beyond this the steps of the multipliers of active rows (divided by
      // slacks near zero) carry no accuracy
      if (muv <= 1e-20) break;
    }
    // predictor: affine target rc = s z (in C.rc)
    build_terms<OCC>(C, sh);
    backward<OCC>(C, sh, true);
    ++*nfact;
    forward<OCC>(C, sh);
    double sigma = 0.0;
    if (m > 0.0) {
      const double aa = row_steps<OCC>(C);
      double sm = 0.0;
      for (int e = lane; e < C.N * C4; e += 64) {
        const int k = e / C4, i = e % C4;
        if (!stance(C, k, i)) continue;
        double sv[NROW], zv[NROW], dsv[NROW], dzv[NROW], cv[NROW];
        ldr(C.s + (size_t)e * NROW, sv);
        ldr(C.z + (size_t)e * NROW, zv);
        ldr(C.ds + (size_t)e * NROW, dsv);
        ldr(C.dz + (size_t)e * NROW, dzv);
        #pragma unroll
        for (int r = 0; r < NROW; ++r) {
          sm += (sv[r] + aa * dsv[r]) * (zv[r] + aa * dzv[r]);
          cv[r] = sv[r] * zv[r] + dsv[r] * dzv[r];   // sigma mu subtracted below
        }
        str(C.rc + (size_t)e * NROW, cv);
      }
      const double mu_aff = wsum(sm) / m;
      sigma = muv > 0.0 ? pow(mu_aff / muv, 3.0) : 0.0;
      // corrector: rc = s z + ds_aff dz_aff - sigma mu, the same Newton matrix
      // (solved with the inverse the predictor's elimination left)
      for (int e = lane; e < C.N * C4; e += 64) {
        const int k = e / C4, i = e % C4;
        if (!stance(C, k, i)) continue;
        gd cv = C.rc + (size_t)e * NROW;
        #pragma unroll
        for (int r = 0; r < NROW; ++r) cv[r] -= sigma * muv;
      }
      // (near the optimum the corrector factors again: the product with the
      // kept inverse carries the Hessian's conditioning into the step, which
      // then limits how closely u meets stationarity)
      build_terms<OCC>(C, sh);
      const bool refactor = muv <= 1e-8;
      backward<OCC>(C, sh, refactor);
      *nfact += refactor;
      forward<OCC>(C, sh);
    }
    const double a = m > 0.0 ? fmin(1.0, 0.99 * row_steps<OCC>(C)) : 1.0;
    // step; residuals and affine target of the new point
    __syncthreads();
    smz = 0.0;
    rpn = 0.0;
    for (int e = lane; e < C.N * U4; e += 64) C.u[e] += a * C.du[e];
    for (int e = lane; e < (C.N + 1) * NX; e += 64) C.x[e] += a * C.dx[e];
    __syncthreads();
    for (int e = lane; e < C.N * C4; e += 64) {
      const int k = e / C4, i = e % C4;
      if (!stance(C, k, i)) continue;
      double u[6], gu[NROW], h[NROW], sc[NROW], sv[NROW], zv[NROW], dsv[NROW], dzv[NROW];
      ld6(C.u + (size_t)k * U4 + 6 * i, u);
      rows_of(C, u, gu, h, sc);
      ldr(C.s + (size_t)e * NROW, sv);
      ldr(C.z + (size_t)e * NROW, zv);
      ldr(C.ds + (size_t)e * NROW, dsv);
      ldr(C.dz + (size_t)e * NROW, dzv);
      #pragma unroll
      for (int r = 0; r < NROW; ++r) {
        sv[r] += a * dsv[r];
        zv[r] += a * dzv[r];
        smz += sv[r] * zv[r];
        rpn = fmax(rpn, fabs((gu[r] - h[r]) / sc[r] + sv[r]));
      }
      str(C.s + (size_t)e * NROW, sv);
      str(C.z + (size_t)e * NROW, zv);
      double cv[NROW];
      #pragma unroll
      for (int r = 0; r < NROW; ++r) cv[r] = sv[r] * zv[r];
      str(C.rc + (size_t)e * NROW, cv);
    }
  }
  *ok = certificate<OCC>(C, sh, res, tol) <= tol;
  return it;
}

template <int OCC>
__global__ void __launch_bounds__(64, OCC) refine_wide_kernel(Problem p, Workspace ws, float* out_u,
                                                         float* out_x, float* out_res,
                                                         int32_t* out_iters, int32_t* out_status,
                                                         int32_t* out_detail, int admm_iters,
                                                         int accel, int refine, int ipm_max,
                                                         double tol) {
  __shared__ WSh sh;
  const int lane = threadIdx.x;
  // the problem's context lives in LDS (the phase functions read its fields
  // with LDS loads, which no wait for a global load in flight holds up)
  __shared__ WCtx C;
  const size_t s0 = (size_t)blockIdx.x * p.n_max;
  if (lane == 0) {
    C.b = blockIdx.x;
    C.n = p.n_max;
    C.N = horizon(p, C.b);
    C.mu = p.mu[C.b];
    C.fz = p.fz_max[C.b];
    C.tm = p.tau_max[C.b];
    C.mg = weight_of(p, C.b);
    C.scf = C.mg;
    C.scm = C.tm > 0.0 ? C.tm : 1.0;
    C.A = (gcf)(p.A + s0 * NX * NX);
    C.B = (gcf)(p.B + s0 * NX * U4);
    C.e = p.e ? (gcf)(p.e + s0 * NX) : nullptr;
    C.x_ref = (gcf)(p.x_ref + s0 * NX);
    C.u_ref = p.u_ref ? (gcf)(p.u_ref + s0 * U4) : nullptr;
    C.x0 = (gcf)(p.x0 + (size_t)C.b * NX);
    C.contact = (const GMEM uint8_t*)(p.contact + s0 * C4);
    carve(C, (gd)(ws.rblk + (size_t)C.b * refine_wide_block_doubles(C.n)));
  }
  __syncthreads();
  if (lane < NX) sh.Q[lane] = p.Q[(size_t)C.b * NX + lane];
  if (lane < U4) sh.R[lane] = p.R[(size_t)C.b * U4 + lane];
  __syncthreads();
  const int N = C.N;

  // input checks as in the two-contact refinement: finiteness of scalars and
  // weights, the bounds, then this problem's stage data
  const int Nraw = horizon_raw(p, C.b);
  int nonfinite = !isfinite(C.mu) || !isfinite(C.fz) || !isfinite(C.tm) || !isfinite(C.mg);
  #pragma unroll
  for (int j = 0; j < NX; ++j) nonfinite |= !isfinite(sh.Q[j]);
  #pragma unroll
  for (int j = 0; j < U4; ++j) nonfinite |= !isfinite(sh.R[j]);
  int bad = 0;
  if (!nonfinite) {
    bad = !(C.mu > 0.0) || !(C.fz >= 0.0) || !(C.tm >= 0.0) || !(C.mg > 0.0) || Nraw < 1 ||
          Nraw > C.n;
    #pragma unroll
    for (int j = 0; j < NX; ++j) bad |= !(sh.Q[j] > 0.0);
    #pragma unroll
    for (int j = 0; j < U4; ++j) bad |= !(sh.R[j] > 0.0);
  }
  if (!bad && !nonfinite) {
    int nf = 0;
    for (int e = lane; e < N * NX * NX; e += 64) nf |= !isfinite(C.A[e]);
    for (int e = lane; e < N * NX * U4; e += 64) nf |= !isfinite(C.B[e]);
    for (int e = lane; e < N * NX; e += 64) {
      nf |= !isfinite(C.x_ref[e]);
      if (C.e) nf |= !isfinite(C.e[e]);
    }
    if (C.u_ref)
      for (int e = lane; e < N * U4; e += 64) nf |= !isfinite(C.u_ref[e]);
    if (lane < NX) nf |= !isfinite(C.x0[lane]);
    if (p.u_prev && lane < U4) nf |= !isfinite(p.u_prev[(size_t)C.b * U4 + lane]);
    nonfinite = wmax((double)nf) > 0.0;
  }
  const size_t ux = (size_t)C.b * C.n * U4, xx = (size_t)C.b * (C.n + 1) * NX;
  if (bad || nonfinite) {
    for (int e = lane; e < C.n * U4; e += 64) out_u[ux + e] = 0.f;
    for (int e = lane; e < (C.n + 1) * NX; e += 64) out_x[xx + e] = 0.f;
    if (lane == 0) {
      if (out_status) out_status[C.b] = bad ? PINMPC_ST_BADINPUT : PINMPC_ST_NONFINITE;
      if (out_iters) out_iters[C.b] = 0;
    }
    if (out_detail && lane < 4) out_detail[(size_t)C.b * 4 + lane] = 0;
    if (out_res && lane < PINMPC_NRES) out_res[(size_t)C.b * PINMPC_NRES + lane] = __builtin_nanf("");
    return;
  }

  // the ADMM point: unscaled inputs of the z iterate, zero on swing contacts
  const float* zsrc = (accel ? ws.cur : ws.hat) + s0 * NSTATE * L4;
  const float tsc = ws.tsc[C.b];
  for (int e = lane; e < N * U4; e += 64) {
    const int k = e / U4, j = e % U4;
    const double sc = (j % 6 < 3) ? (double)ws.sf[s0 + k] : (double)tsc;
    const double v = (double)zsrc[(size_t)k * NSTATE * L4 + NX + j] * sc;
    C.u[e] = stance(C, k, j / 6) ? v : 0.0;
  }
  double res[PINMPC_NRES] = {0, 0, 0, 0, 0};
  int its = 0, nfact = 0;
  bool ok = false;
  (void)rollout<OCC>(C, sh);
  if (refine) {
    its = ipm<OCC>(C, sh, ipm_max, tol, res, &ok, &nfact);   // res: the returned point's
  } else {
    // the ADMM point as it is
    (void)certificate<OCC>(C, sh, res, tol);
  }

  // outputs
  __syncthreads();
  for (int e = lane; e < C.n * U4; e += 64) out_u[ux + e] = (e < N * U4) ? (float)C.u[e] : 0.f;
  for (int e = lane; e < (C.n + 1) * NX; e += 64)
    out_x[xx + e] = (e < (N + 1) * NX) ? (float)C.x[e] : 0.f;
  if (lane == 0) {
    atomicAdd(ws.work, (unsigned long long)its * (unsigned long long)N);
    if (out_status)
      out_status[C.b] = refine ? (ok ? PINMPC_ST_OK : PINMPC_ST_UNPOLISHED) : PINMPC_ST_MAXITER;
    if (out_iters) out_iters[C.b] = admm_iters + its;
  }
  if (out_detail && lane < 4) {
    const int v = lane == 1 ? its : lane == 2 ? nfact * N : lane == 3 ? 1 : 0;
    out_detail[(size_t)C.b * 4 + lane] = v;
  }
  if (out_res && lane < PINMPC_NRES) out_res[(size_t)C.b * PINMPC_NRES + lane] = (float)res[lane];
}

}  // namespace

hipError_t launch_refine_wide(const Problem& p, const Workspace& w, const pinmpc_settings& s,
                              const pinmpc_out& out, hipStream_t st) {
  if (p.batch == 0) return hipSuccess;
  if (p.nc != C4 || p.n_max > PINMPC_NMAX) return hipErrorInvalidValue;
  // two waves per SIMD once the batch has more problems than the chip has
  // SIMDs; below that every problem has a SIMD of its own and the one-wave
  // build, with all registers for its stage, is faster (both builds do the
  // same arithmetic in the same order: bitwise the same results)
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  if (p.batch > 4 * cus)
    hipLaunchKernelGGL(refine_wide_kernel<2>, dim3(p.batch), dim3(64), 0, st, p, w, out.u, out.x,
                       out.res, out.iters, out.status, out.detail, s.iters, s.accel, s.refine,
                       s.ipm_iters, s.kkt_tol);
  else
    hipLaunchKernelGGL(refine_wide_kernel<1>, dim3(p.batch), dim3(64), 0, st, p, w, out.u, out.x,
                       out.res, out.iters, out.status, out.detail, s.iters, s.accel, s.refine,
                       s.ipm_iters, s.kkt_tol);
  return hipGetLastError();
}

}  // namespace pinmpc
