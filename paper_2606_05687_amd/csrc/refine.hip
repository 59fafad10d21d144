// FP64 refinement and certification of the ADMM result, one 64-lane wave per
// problem (problems are independent, so each wave runs its own loop).
//
// The ADMM of Sec. III reaches the QP optimum only in the limit; its last
// projection fixes a guess of the active faces of every contact's wrench set.
// From that guess the kernel runs, all in FP64:
//  A. active-set passes: solve the equality-constrained LQ problem with each
//     contact's input restricted to the affine hull of its face (Riccati
//     recursion over the horizon with u_k = c_k + P_k w_k), evaluate the KKT
//     residuals with costates from the adjoint recursion and row multipliers
//     from the face, and update the faces by the primal-dual active-set rule
//     (row active iff mu_i s_i + (G_i u - h_i) > 0); stop when certified, when
//     the face set repeats, or after refine_passes passes;
//  B. if not certified: a primal-dual interior point with Mehrotra's
//     predictor-corrector on the same QP (each Newton step a Riccati recursion
//     with input Hessian R + G^T diag(z/s) G), then faces from z > s and
//  C. active-set passes again from those faces (polish_passes).
// The returned u is the last equality-constrained solution, x its rollout in
// FP64, and res the normalised residuals (r_dyn, r_ineq, r_stat, r_comp,
// r_sign) of that point.
#include "pinmpc_internal.h"

namespace pinmpc {

namespace {

constexpr int W64 = 64;
constexpr int GJW = NU + NX + 1 + NU;   // 38 columns of the augmented system

// One problem's view: its inputs and its FP64 scratch block, all as
// pointers to the problem's own first stage, so stage k is plain k.
struct Ctx {
  int b, N, n;
  double mu, fz, tm, mg;
  const double* Q;   // LDS copies of the diagonal weights
  const double* R;
  const float *A, *B, *e, *x_ref, *u_ref, *x0;
  const uint8_t* contact;
  double *rK, *rkap, *rL, *rHwx, *ru, *rx, *rlam, *rg, *rmu, *rs, *rz, *rds, *rdz, *rdu, *rdx;
  double* ftab;   // [n][2][18] face tables: force projector 3x3, force offset,
                  // moment projector diagonal, moment offset
  double* wrow;   // [n][2][11] interior-point row weights z / (s sc^2)
  double* crow;   // [n][2][11] interior-point row coefficients of the linear term
  int32_t* faces;
};

// ------------------------------------------------------------ small helpers

// The refinement runs one 64-lane wave per workgroup.  LDS operations of a
// wave execute in issue order, so handing data between the lanes of the wave
// through LDS needs only a point the compiler does not move memory accesses
// across (wsync).  Global memory written by one lane and read by another needs
// the workgroup barrier with its memory fence (gsync); it is used where one
// phase's global outputs feed the next phase, not inside the stage loops.
__device__ inline void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}
__device__ inline void gsync() { __syncthreads(); }

__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline uint64_t wave_xor(uint64_t v) {
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t lo = __shfl_xor((uint32_t)v, o, 64);
    const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), o, 64);
    v ^= ((uint64_t)hi << 32) | lo;
  }
  return v;
}

// Row i (0..10) of one stance contact's wrench constraints on (f, tau).
__device__ inline void wrench_row(int i, double mu, double fz, double tm, double g[6],
                                  double* h) {
  for (int a = 0; a < 6; ++a) g[a] = 0.0;
  switch (i) {
    case 0: g[0] = 1; g[2] = -mu; *h = 0; break;
    case 1: g[0] = -1; g[2] = -mu; *h = 0; break;
    case 2: g[1] = 1; g[2] = -mu; *h = 0; break;
    case 3: g[1] = -1; g[2] = -mu; *h = 0; break;
    case 4: g[2] = 1; *h = fz; break;
    default: {
      const int a = (i - 5) % 3;
      g[3 + a] = (i < 8) ? 1.0 : -1.0;
      *h = tm;
    }
  }
}

__device__ inline bool face_apex(int code) {
  const int f = code & 31;
  return ((f & 3) == 3) || ((f & 12) == 12);
}

// Force rows of the pyramid as fixed vectors: row i (0..4) is g_i^T f <= h_i.
__device__ inline void force_row(int i, double mu, double g[3]) {
  g[0] = (i == 0) ? 1.0 : (i == 1 ? -1.0 : 0.0);
  g[1] = (i == 2) ? 1.0 : (i == 3 ? -1.0 : 0.0);
  g[2] = (i < 4) ? -mu : 1.0;
}

// Solve the 5 x 5 system M y = r in place (Gauss-Jordan, no pivoting; M is
// SPD on the active rows and the identity on the others).  All indices are
// compile-time after unrolling, so the arrays stay in registers.
__device__ inline void solve5(double M[5][5], double r[5]) {
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    const double inv = 1.0 / M[j][j];
#pragma unroll
    for (int c = 0; c < 5; ++c) M[j][c] *= inv;
    r[j] *= inv;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      if (i == j) continue;
      const double f = M[i][j];
#pragma unroll
      for (int c = 0; c < 5; ++c) M[i][c] -= f * M[j][c];
      r[i] -= f * r[j];
    }
  }
}

// Masked Gram system of the active force rows: (G_A G_A^T) on active rows,
// identity elsewhere.
__device__ inline void gram5(int mask, double mu, double M[5][5]) {
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    double gi[3];
    force_row(i, mu, gi);
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      double gj[3];
      force_row(j, mu, gj);
      const bool ai = (mask >> i) & 1, aj = (mask >> j) & 1;
      M[i][j] = (ai && aj) ? gi[0] * gj[0] + gi[1] * gj[1] + gi[2] * gj[2] : (i == j ? 1.0 : 0.0);
    }
  }
}

// Affine hull of a contact's face: projector P (6x6, block diagonal) and a
// point c with u = c + P w spanning the face.  For the force block with
// active rows A (independent unless the face is the apex):
//   P = I - G_A^T (G_A G_A^T)^{-1} G_A,   c = G_A^T (G_A G_A^T)^{-1} h_A.
__device__ void face_affine(int code, double mu, double fz, double tm, double P[6][6],
                            double c[6]) {
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    c[a] = 0.0;
#pragma unroll
    for (int b = 0; b < 6; ++b) P[a][b] = 0.0;
  }
  if (!face_apex(code)) {
    const int mask = code & 31;
    double M[5][5], y[5];
    gram5(mask, mu, M);
#pragma unroll
    for (int i = 0; i < 5; ++i) y[i] = ((mask >> i) & 1) && i == 4 ? fz : 0.0;
    // columns of (G G^T)^{-1} G, one solve per coordinate, and the point c
    double Gi[5][3];
#pragma unroll
    for (int col = 0; col < 3; ++col) {
      double Mc[5][5], r[5];
#pragma unroll
      for (int i = 0; i < 5; ++i) {
#pragma unroll
        for (int j = 0; j < 5; ++j) Mc[i][j] = M[i][j];
        double gi[3];
        force_row(i, mu, gi);
        r[i] = ((mask >> i) & 1) ? gi[col] : 0.0;
      }
      solve5(Mc, r);
#pragma unroll
      for (int i = 0; i < 5; ++i) Gi[i][col] = r[i];
    }
    solve5(M, y);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double ca = 0.0;
#pragma unroll
      for (int i = 0; i < 5; ++i) {
        double gi[3];
        force_row(i, mu, gi);
        if ((mask >> i) & 1) ca += gi[a] * y[i];
      }
      c[a] = ca;
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        double t = (a == b) ? 1.0 : 0.0;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
          double gi[3];
          force_row(i, mu, gi);
          if ((mask >> i) & 1) t -= gi[a] * Gi[i][b];
        }
        P[a][b] = t;
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (code >> (8 + a) & 1) c[3 + a] = tm;
    else if (code >> (11 + a) & 1) c[3 + a] = -tm;
    else P[3 + a][3 + a] = 1.0;
  }
}

// Input blocks: force triples (3 x 3) and single moment components.  Face
// projectors P_k and the interior-point input Hessian R' are block diagonal
// in these blocks, so products with them only run over the block of the
// column (exact, not an approximation).
__device__ inline int blk_start(int j) { return (j % 6 < 3) ? j - j % 6 : j; }
__device__ inline int blk_len(int j) { return (j % 6 < 3) ? 3 : 1; }

// --------------------------------------------------------------- LDS state

struct Sh {
  double S[NX * NX], s[NX];           // value function of x_{k+1}
  double A[NX * NX], B[NX * NU];
  double W[NX * NX], WA[NX * NX];
  double P[NU * NU], c[NU], Rp[NU * NU];
  double Bp[NX * NU], WBp[NX * NU];
  double Hwx[NU * NX], K[NU * NX];
  double om[NX], d[NX], Wdo[NX], hw[NU], kap[NU], rho[NU], q[NX];
  double xv[NX], wv[NU], uv[NU], xn[NX];
  double G[NU * GJW];                 // Gauss-Jordan augmented [H | Hwx | hw | I]
  double fac[16];
  double Qd[NX], Rd[NU];              // diagonal weights of the problem
};

__device__ inline void load_AB(const Ctx& C, Sh& sh, int k) {
  const int lane = threadIdx.x;
  const float* A = C.A + k * NX * NX;
  const float* B = C.B + k * NX * NU;
  for (int i = lane; i < NX * NX; i += W64) sh.A[i] = (double)A[i];
  for (int i = lane; i < NX * NU; i += W64) sh.B[i] = (double)B[i];
}

constexpr int FT = 18;   // doubles per contact in the face table

// Face tables of every (stage, contact) of the problem, computed in parallel
// over (stage, contact) once per equality-constrained pass.
__device__ void build_face_table(const Ctx& C) {
  const int lane = threadIdx.x;
  for (int e = lane; e < C.N * 2; e += W64) {
    const int k = e >> 1, i = e & 1;
    double* t = C.ftab + (size_t)e * FT;
    if (C.contact[k * 2 + i]) {
      double P6[6][6], c6[6];
      face_affine(C.faces[k * 2 + i], C.mu, C.fz, C.tm, P6, c6);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int b = 0; b < 3; ++b) t[a * 3 + b] = P6[a][b];
        t[9 + a] = c6[a];
        t[12 + a] = P6[3 + a][3 + a];
        t[15 + a] = c6[3 + a];
      }
    } else {
#pragma unroll
      for (int a = 0; a < FT; ++a) t[a] = 0.0;
    }
  }
}

// Face projector/offset of stage k into sh.P, sh.c, filled in parallel from
// the face table (equality passes) or as the stance mask (Newton steps).
__device__ inline void load_face(const Ctx& C, Sh& sh, int k, bool newton) {
  const int lane = threadIdx.x;
  for (int e = lane; e < NU * NU; e += W64) {
    const int r = e / NU, c = e % NU;
    const int i = r / 6;
    double v = 0.0;
    if (i == c / 6 && C.contact[k * 2 + i]) {
      const int a = r % 6, b = c % 6;
      if (newton) {
        v = (a == b) ? 1.0 : 0.0;
      } else {
        const double* t = C.ftab + ((size_t)k * 2 + i) * FT;
        if (a < 3 && b < 3) v = t[a * 3 + b];
        else if (a == b) v = t[12 + a - 3];
      }
    }
    sh.P[e] = v;
  }
  if (lane < NU) {
    const int i = lane / 6, a = lane % 6;
    double v = 0.0;
    if (!newton && C.contact[k * 2 + i]) {
      const double* t = C.ftab + ((size_t)k * 2 + i) * FT;
      v = (a < 3) ? t[9 + a] : t[15 + a - 3];
    }
    sh.c[lane] = v;
  }
  wsync();
}

// Interior-point row terms of every stance row, in parallel over rows:
// the weight z / (s sc^2) of the input Hessian and the coefficient
// z + (-rc + z rp) / s of the linear term (rows scaled by sc).
__device__ void build_row_terms(const Ctx& C, const double* rcvec) {
  const int lane = threadIdx.x;
  for (int e = lane; e < C.N * 2 * NROW; e += W64) {
    const int k = e / (2 * NROW), i = (e / NROW) & 1, r = e % NROW;
    if (!C.contact[k * 2 + i]) {
      C.wrow[e] = 0.0;
      C.crow[e] = 0.0;
      continue;
    }
    double g[6], h;
    wrench_row(r, C.mu, C.fz, C.tm, g, &h);
    const double sc = (r < 5) ? C.mg : C.tm;
    double gu = 0.0;
#pragma unroll
    for (int t = 0; t < 6; ++t) gu += g[t] * C.ru[k * NU + 6 * i + t];
    const double s = C.rs[e], z = C.rz[e];
    const double rp = (gu - h) / sc + s;
    C.wrow[e] = z / s / (sc * sc);
    C.crow[e] = (z + (-rcvec[e] + z * rp) / s) / sc;
  }
}

// ------------------------------------------------------ Riccati recursion
//
// Solves   min sum_k 1/2 x_{k+1}^T Q x_{k+1} + q_k^T x_{k+1}
//                    + 1/2 u_k^T R'_k u_k + rho_k^T u_k
//          s.t. x_{k+1} = A_k x_k + B_k u_k + e_k,  u_k = c_k + P_k w_k
// (P_k an orthogonal projector) by the backward recursion on the value
// function V(x) = 1/2 x^T S x + s^T x and the forward rollout.
//   newton = false: the equality-constrained tracking problem of the faces
//                   (q = -Q r, rho = -R u_ref, R' = R, e from the data);
//   newton = true:  the interior-point Newton step, x_0 = 0, e = 0,
//                   q = Q (x_{k+1} - r), R' = R + G^T diag(z/s) G,
//                   rho from ipm_rho (stage inputs), P = stance mask.
// With factor = false only the linear part is recomputed from the stored
// factors (second right-hand side of the same Newton matrix).

enum class Mode { EQ, NEWTON };

__device__ void stage_rp(const Ctx& C, Sh& sh, int k, Mode mode) {
  // R'_k = R (+ sum over stance rows of w_r g_r g_r^T in Newton steps), in
  // parallel over the entries of the two 6 x 6 contact blocks
  const int lane = threadIdx.x;
  for (int e = lane; e < NU * NU; e += W64) {
    const int r = e / NU, c = e % NU;
    double v = (r == c) ? C.R[r] : 0.0;
    const int i = r / 6;
    if (mode == Mode::NEWTON && i == c / 6 && C.contact[k * 2 + i]) {
      const int a = r % 6, b = c % 6;
      const double* w = C.wrow + ((size_t)k * 2 + i) * NROW;
#pragma unroll
      for (int row = 0; row < NROW; ++row) {
        double g[6], h;
        wrench_row(row, C.mu, C.fz, C.tm, g, &h);
        v += w[row] * g[a] * g[b];
      }
    }
    sh.Rp[e] = v;
  }
  wsync();
}

// Linear input term rho_k of stage k into sh.rho.
__device__ void stage_rho(const Ctx& C, Sh& sh, int k, Mode mode) {
  const int lane = threadIdx.x;
  if (lane < NU) {
    const int j = lane;
    const double ur = C.u_ref ? (double)C.u_ref[k * NU + j] : 0.0;
    double r;
    if (mode == Mode::EQ) {
      r = -C.R[j] * ur;
    } else {
      r = C.R[j] * (C.ru[k * NU + j] - ur);
      const int i = j / 6, a = j % 6;
      if (C.contact[k * 2 + i]) {
        const double* cr = C.crow + ((size_t)k * 2 + i) * NROW;
#pragma unroll
        for (int row = 0; row < NROW; ++row) {
          double g[6], h;
          wrench_row(row, C.mu, C.fz, C.tm, g, &h);
          r += g[a] * cr[row];
        }
      }
    }
    sh.rho[j] = r;
  }
}

__device__ void riccati(const Ctx& C, Sh& sh, Mode mode, bool factor, const double* rcvec) {
  gsync();
  if (mode == Mode::EQ) build_face_table(C);
  else build_row_terms(C, rcvec);
  gsync();
  const int lane = threadIdx.x;
  const int N = C.N;
  for (int i = lane; i < NX * NX; i += W64) sh.S[i] = 0.0;
  if (lane < NX) sh.s[lane] = 0.0;
  wsync();
  for (int k = N - 1; k >= 0; --k) {
    const int st = k;
    load_AB(C, sh, k);
    load_face(C, sh, k, mode == Mode::NEWTON);
    if (factor) stage_rp(C, sh, k, mode);
    stage_rho(C, sh, k, mode);
    if (lane < NX) {
      const double r = (double)C.x_ref[st * NX + lane];
      double q;
      if (mode == Mode::EQ) q = -C.Q[lane] * r;
      else q = C.Q[lane] * (C.rx[(k + 1) * NX + lane] - r);
      sh.om[lane] = q + sh.s[lane];
    }
    wsync();
    // Bp = B P ; d = B c + e
    for (int e = lane; e < NX * NU; e += W64) {
      const int i = e / NU, j = e % NU;
      const int l0 = blk_start(j), l1 = l0 + blk_len(j);
      double acc = 0.0;
      for (int l = l0; l < l1; ++l) acc += sh.B[i * NU + l] * sh.P[l * NU + j];
      sh.Bp[e] = acc;
    }
    if (lane < NX) {
      double acc = 0.0;
      if (mode == Mode::EQ) {
        for (int l = 0; l < NU; ++l) acc += sh.B[lane * NU + l] * sh.c[l];
        if (C.e) acc += (double)C.e[st * NX + lane];
      }
      sh.d[lane] = acc;
    }
    if (factor) {
      for (int e = lane; e < NX * NX; e += W64)
        sh.W[e] = sh.S[e] + ((e % (NX + 1) == 0) ? C.Q[e / NX] : 0.0);
    }
    wsync();
    if (factor) {
      // WA, WBp
      for (int e = lane; e < NX * NX + NX * NU; e += W64) {
        if (e < NX * NX) {
          const int i = e / NX, j = e % NX;
          double acc = 0.0;
          for (int l = 0; l < NX; ++l) acc += sh.W[i * NX + l] * sh.A[l * NX + j];
          sh.WA[e] = acc;
        } else {
          const int f = e - NX * NX, i = f / NU, j = f % NU;
          double acc = 0.0;
          for (int l = 0; l < NX; ++l) acc += sh.W[i * NX + l] * sh.Bp[l * NU + j];
          sh.WBp[f] = acc;
        }
      }
    }
    wsync();
    if (lane < NX) {
      // W d + omega (W = Q + S)
      double acc = sh.om[lane];
      if (mode == Mode::EQ)
        for (int l = 0; l < NX; ++l)
          acc += (sh.S[lane * NX + l] + (l == lane ? C.Q[lane] : 0.0)) * sh.d[l];
      sh.Wdo[lane] = acc;
    }
    if (factor) {
      // T = R' P, held in K until K itself is formed
      for (int e = lane; e < NU * NU; e += W64) {
        const int i = e / NU, j = e % NU;
        const int l0 = blk_start(j), l1 = l0 + blk_len(j);
        double acc = 0.0;
        if (blk_start(i) == l0)
          for (int l = l0; l < l1; ++l) acc += sh.Rp[i * NU + l] * sh.P[l * NU + j];
        sh.K[e] = acc;   // scratch
      }
    }
    wsync();
    if (factor) {
      // H = P R' P + Bp^T W Bp + (I - P) ; Hwx = Bp^T W A, straight into the
      // augmented Gauss-Jordan system [H | Hwx | hw | I]
      for (int e = lane; e < NU * NU + NU * NX; e += W64) {
        if (e < NU * NU) {
          const int i = e / NU, j = e % NU;
          double acc = ((i == j) ? 1.0 : 0.0) - sh.P[i * NU + j];
          const int l0 = blk_start(i), l1 = l0 + blk_len(i);
          if (blk_start(j) == l0)
            for (int l = l0; l < l1; ++l) acc += sh.P[l * NU + i] * sh.K[l * NU + j];
          for (int l = 0; l < NX; ++l) acc += sh.Bp[l * NU + i] * sh.WBp[l * NU + j];
          sh.G[i * GJW + j] = acc;
          if (mode == Mode::NEWTON) sh.G[i * GJW + NU + NX + 1 + j] = (i == j) ? 1.0 : 0.0;
        } else {
          const int f = e - NU * NU, i = f / NX, j = f % NX;
          double acc = 0.0;
          for (int l = 0; l < NX; ++l) acc += sh.Bp[l * NU + i] * sh.WA[l * NX + j];
          sh.Hwx[f] = acc;
          sh.G[i * GJW + NU + j] = acc;
        }
      }
    } else {
      for (int e = lane; e < NU * NX; e += W64) sh.Hwx[e] = C.rHwx[st * NU * NX + e];
    }
    if (lane < NU) {
      // hw = P (R' c + rho) + Bp^T (W d + omega)
      double acc = 0.0;
      const int l0 = blk_start(lane), l1 = l0 + blk_len(lane);
      for (int l = l0; l < l1; ++l) {
        double t = sh.rho[l];
        if (mode == Mode::EQ)
          for (int m = l0; m < l1; ++m) t += sh.Rp[l * NU + m] * sh.c[m];
        acc += sh.P[lane * NU + l] * t;
      }
      for (int l = 0; l < NX; ++l) acc += sh.Bp[l * NU + lane] * sh.Wdo[l];
      sh.hw[lane] = acc;
      if (factor) sh.G[lane * GJW + NU + NX] = acc;
    }
    wsync();
    if (factor) {
      // Gauss-Jordan elimination (H is SPD: no pivoting) over all 64 lanes:
      // afterwards G = [I | H^{-1} Hwx | H^{-1} hw | H^{-1}]; the equality
      // pass needs no explicit inverse, so it stops at column 25.
      const int gw = (mode == Mode::NEWTON) ? GJW : NU + NX + 1;
      for (int j = 0; j < NU; ++j) {
        const double piv = sh.G[j * GJW + j];
        wsync();
        for (int c = j + lane; c < gw; c += W64) sh.G[j * GJW + c] /= piv;
        wsync();
        if (lane < NU) sh.fac[lane] = sh.G[lane * GJW + j];
        wsync();
        for (int e = lane; e < NU * (gw - j - 1); e += W64) {
          const int r = e / (gw - j - 1), c = j + 1 + e % (gw - j - 1);
          if (r != j) sh.G[r * GJW + c] -= sh.fac[r] * sh.G[j * GJW + c];
        }
        wsync();
      }
      for (int e = lane; e < NU * NX; e += W64) {
        const int i = e / NX, j = e % NX;
        sh.K[e] = -sh.G[i * GJW + NU + j];
      }
      if (lane < NU) sh.kap[lane] = -sh.G[lane * GJW + NU + NX];
      // keep H^{-1} and Hwx for a second right-hand side of the same matrix
      if (mode == Mode::NEWTON) {
        double* Hi = C.rL + st * NU * NU;
        for (int e = lane; e < NU * NU; e += W64)
          Hi[e] = sh.G[(e / NU) * GJW + NU + NX + 1 + e % NU];
        for (int e = lane; e < NU * NX; e += W64) C.rHwx[st * NU * NX + e] = sh.Hwx[e];
      }
    } else {
      const double* Hi = C.rL + st * NU * NU;
      if (lane < NU) {
        double acc = 0.0;
        for (int l = 0; l < NU; ++l) acc += Hi[lane * NU + l] * sh.hw[l];
        sh.kap[lane] = -acc;
      }
      for (int e = lane; e < NU * NX; e += W64) sh.K[e] = C.rK[st * NU * NX + e];
    }
    wsync();
    if (factor)
      for (int e = lane; e < NU * NX; e += W64) C.rK[st * NU * NX + e] = sh.K[e];
    if (lane < NU) C.rkap[st * NU + lane] = sh.kap[lane];
    // S = A^T W A + Hwx^T K ; s = A^T (W d + omega) + Hwx^T kap
    if (factor) {
      // upper triangle of the (symmetric) new S, mirrored below
      for (int e = lane; e < NX * (NX + 1) / 2; e += W64) {
        int i = 0, rem = e;
        while (rem >= NX - i) { rem -= NX - i; ++i; }
        const int j = i + rem;
        double acc = 0.0;
        for (int l = 0; l < NX; ++l) acc += sh.A[l * NX + i] * sh.WA[l * NX + j];
        for (int l = 0; l < NU; ++l) acc += sh.Hwx[l * NX + i] * sh.K[l * NX + j];
        sh.W[i * NX + j] = acc;    // new S, copied below
      }
    }
    if (lane < NX) {
      double acc = 0.0;
      for (int l = 0; l < NX; ++l) acc += sh.A[l * NX + lane] * sh.Wdo[l];
      for (int l = 0; l < NU; ++l) acc += sh.Hwx[l * NX + lane] * sh.kap[l];
      sh.xn[lane] = acc;
    }
    wsync();
    if (factor)
      for (int e = lane; e < NX * NX; e += W64) {
        const int i = e / NX, j = e % NX;
        sh.S[e] = (i <= j) ? sh.W[i * NX + j] : sh.W[j * NX + i];
      }
    if (lane < NX) sh.s[lane] = sh.xn[lane];
    wsync();
  }
  // forward rollout (reads the gains written by other lanes above)
  gsync();
  if (lane < NX) {
    sh.xv[lane] = (mode == Mode::EQ) ? (double)C.x0[lane] : 0.0;
  }
  wsync();
  double* xout = (mode == Mode::EQ) ? C.rx : C.rdx;
  double* uout = (mode == Mode::EQ) ? C.ru : C.rdu;
  if (lane < NX) xout[0 + lane] = sh.xv[lane];
  for (int k = 0; k < N; ++k) {
    const int st = k;
    load_AB(C, sh, k);
    load_face(C, sh, k, mode == Mode::NEWTON);
    if (lane < NU) {
      double acc = C.rkap[st * NU + lane];
      for (int l = 0; l < NX; ++l) acc += C.rK[st * NU * NX + lane * NX + l] * sh.xv[l];
      sh.wv[lane] = acc;
    }
    wsync();
    if (lane < NU) {
      double acc = sh.c[lane];
      for (int l = 0; l < NU; ++l) acc += sh.P[lane * NU + l] * sh.wv[l];
      sh.uv[lane] = acc;
      uout[st * NU + lane] = acc;
    }
    wsync();
    if (lane < NX) {
      double acc = 0.0;
      for (int l = 0; l < NX; ++l) acc += sh.A[lane * NX + l] * sh.xv[l];
      for (int l = 0; l < NU; ++l) acc += sh.B[lane * NU + l] * sh.uv[l];
      if (mode == Mode::EQ && C.e) acc += (double)C.e[st * NX + lane];
      sh.xn[lane] = acc;
    }
    wsync();
    if (lane < NX) {
      sh.xv[lane] = sh.xn[lane];
      xout[(k + 1) * NX + lane] = sh.xn[lane];
    }
    wsync();
  }
  gsync();
}

// Costates p_{k+1} = Q (x_{k+1} - r_k) + A_{k+1}^T p_{k+2} and the reduced
// gradient g_k = R (u_k - u_ref_k) + B_k^T p_{k+1}.
__device__ void costates_grad(const Ctx& C, Sh& sh) {
  gsync();
  const int lane = threadIdx.x;
  for (int k = C.N - 1; k >= 0; --k) {
    const int st = k;
    if (lane < NX) {
      const double x = C.rx[(k + 1) * NX + lane];
      double acc = C.Q[lane] * (x - (double)C.x_ref[st * NX + lane]);
      if (k + 1 < C.N) {
        const float* A1 = C.A + (st + 1) * NX * NX;
        for (int l = 0; l < NX; ++l) acc += (double)A1[l * NX + lane] * sh.xn[l];
      }
      sh.om[lane] = acc;
    }
    wsync();
    if (lane < NX) {
      sh.xn[lane] = sh.om[lane];
      C.rlam[st * NX + lane] = sh.om[lane];
    }
    wsync();
  }
  gsync();
  for (int e = lane; e < C.N * NU; e += W64) {
    const int k = e / NU, j = e % NU;
    const int st = k;
    const float* B = C.B + st * NX * NU;
    const double ur = C.u_ref ? (double)C.u_ref[st * NU + j] : 0.0;
    double acc = C.R[j] * (C.ru[st * NU + j] - ur);
    for (int l = 0; l < NX; ++l) acc += (double)B[l * NU + j] * C.rlam[st * NX + l];
    C.rg[st * NU + j] = acc;
  }
  gsync();
}

// Row multipliers of each stance contact from its face and the gradient, and
// the normalised KKT residuals of the current (u, x, p, mu).  Returns KKT.
__device__ double multipliers_kkt(const Ctx& C, double res[PINMPC_NRES]) {
  gsync();
  const int lane = threadIdx.x;
  double r_ineq = 0.0, stat = 0.0, term = 0.0, comp = 0.0, mumax = 0.0, neg = 0.0;
  for (int e = lane; e < C.N * 2; e += W64) {
    const int k = e >> 1, i = e & 1;
    const int st = k;
    const double* u = C.ru + st * NU + 6 * i;
    const double* g = C.rg + st * NU + 6 * i;
    double* mu = C.rmu + (st * 2 + i) * NROW;
    for (int r = 0; r < NROW; ++r) mu[r] = 0.0;
    if (!C.contact[st * 2 + i]) {
      for (int a = 0; a < 6; ++a) r_ineq = fmax(r_ineq, fabs(u[a]) / C.mg);
      continue;
    }
    const int code = C.faces[st * 2 + i];
    for (int a = 0; a < 6; ++a) {
      const double ur = C.u_ref ? (double)C.u_ref[st * NU + 6 * i + a] : 0.0;
      const double ru = C.R[6 * i + a] * (u[a] - ur);
      term = fmax(term, fmax(fabs(ru), fabs(g[a] - ru)));
    }
    // force multipliers: G_A^T mu_A = -g_f on the face's rows (least squares
    // through the masked Gram system); at the apex the four side rows are
    // dependent, so take the three-row subset whose multipliers are most
    // nonnegative (some subset is nonnegative exactly when -g_f lies in the
    // normal cone of the apex)
    if (face_apex(code)) {
      double best = -1e300, bm[5] = {0, 0, 0, 0, 0};
#pragma unroll
      for (int drop = 0; drop < 4; ++drop) {
        const int mask = 15 & ~(1 << drop);
        double M[5][5], r[5];
        gram5(mask, C.mu, M);
#pragma unroll
        for (int i = 0; i < 5; ++i) {
          double gi[3];
          force_row(i, C.mu, gi);
          r[i] = ((mask >> i) & 1) ? -(gi[0] * g[0] + gi[1] * g[1] + gi[2] * g[2]) : 0.0;
        }
        solve5(M, r);
        double mn = 1e300;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if ((mask >> i) & 1) mn = fmin(mn, r[i]);
        if (mn > best) {
          best = mn;
#pragma unroll
          for (int i = 0; i < 5; ++i) bm[i] = ((mask >> i) & 1) ? r[i] : 0.0;
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) mu[i] = bm[i];
    } else {
      const int mask = code & 31;
      if (mask) {
        double M[5][5], r[5];
        gram5(mask, C.mu, M);
#pragma unroll
        for (int i = 0; i < 5; ++i) {
          double gi[3];
          force_row(i, C.mu, gi);
          r[i] = ((mask >> i) & 1) ? -(gi[0] * g[0] + gi[1] * g[1] + gi[2] * g[2]) : 0.0;
        }
        solve5(M, r);
#pragma unroll
        for (int i = 0; i < 5; ++i)
          if ((mask >> i) & 1) mu[i] = r[i];
      }
    }
    for (int a = 0; a < 3; ++a) {
      if (code >> (8 + a) & 1) mu[5 + a] = -g[3 + a];
      else if (code >> (11 + a) & 1) mu[8 + a] = g[3 + a];
    }
    // residual pieces
    double gm[6] = {0, 0, 0, 0, 0, 0};
    for (int r = 0; r < NROW; ++r) {
      double gg[6], hh;
      wrench_row(r, C.mu, C.fz, C.tm, gg, &hh);
      double gu = 0.0;
      for (int a = 0; a < 6; ++a) {
        gu += gg[a] * u[a];
        gm[a] += gg[a] * mu[r];
      }
      r_ineq = fmax(r_ineq, fmax(0.0, gu - hh) / C.mg);
      comp = fmax(comp, mu[r] * fmax(0.0, hh - gu));
      mumax = fmax(mumax, mu[r]);
      neg = fmax(neg, -mu[r]);
    }
    for (int a = 0; a < 6; ++a) {
      term = fmax(term, fabs(gm[a]));
      stat = fmax(stat, fabs(g[a] + gm[a]));
    }
  }
  // state-side term norms: |Q (x - r)|, |p|, |A^T p| = |p_k - Q(x_{k+1} - r_k)|
  for (int e = lane; e < C.N * NX; e += W64) {
    const int k = e / NX, j = e % NX;
    const int st = k;
    const double x = C.rx[(k + 1) * NX + j];
    const double qx = C.Q[j] * (x - (double)C.x_ref[st * NX + j]);
    const double lam = C.rlam[st * NX + j];
    term = fmax(term, fmax(fabs(qx), fmax(fabs(lam), fabs(lam - qx))));
  }
  r_ineq = wave_max(r_ineq);
  stat = wave_max(stat);
  term = wave_max(term);
  comp = wave_max(comp);
  mumax = wave_max(mumax);
  neg = wave_max(neg);
  res[0] = 0.0;   // r_dyn: filled by the caller from the rollout
  res[1] = r_ineq;
  res[2] = stat / (1.0 + term);
  res[3] = comp / (1.0 + mumax * C.mg);
  res[4] = fmax(0.0, neg) / (1.0 + term);
  double kkt = 0.0;
  for (int i = 1; i < PINMPC_NRES; ++i) kkt = fmax(kkt, res[i]);
  return kkt;
}

// Dynamics residual of the FP64 trajectory (rx, ru).
__device__ double dyn_residual(const Ctx& C) {
  gsync();
  const int lane = threadIdx.x;
  double r = 0.0;
  for (int e = lane; e < C.N * NX; e += W64) {
    const int k = e / NX, i = e % NX;
    const int st = k;
    const double* x = C.rx + k * NX;
    const float* A = C.A + st * NX * NX + i * NX;
    const float* B = C.B + st * NX * NU + i * NU;
    double ax = 0.0, bu = 0.0;
    for (int l = 0; l < NX; ++l) ax += (double)A[l] * x[l];
    for (int l = 0; l < NU; ++l) bu += (double)B[l] * C.ru[st * NU + l];
    const double ee = C.e ? (double)C.e[st * NX + i] : 0.0;
    const double d = x[NX + i] - ax - bu - ee;
    const double den = 1.0 + fmax(fabs(x[NX + i]), fmax(fabs(ax), fabs(bu)));
    r = fmax(r, fabs(d) / den);
  }
  return wave_max(r);
}

// Primal-dual active-set update of the faces; returns an order-independent
// hash of the new face set.
__device__ uint64_t pdas_update(const Ctx& C) {
  gsync();
  const int lane = threadIdx.x;
  uint64_t hsh = 0;
  for (int e = lane; e < C.N * 2; e += W64) {
    const int k = e >> 1, i = e & 1;
    const int st = k;
    int code = 0;
    if (C.contact[st * 2 + i]) {
      const double* u = C.ru + st * NU + 6 * i;
      const double* mu = C.rmu + (st * 2 + i) * NROW;
      for (int r = 0; r < NROW; ++r) {
        double gg[6], hh;
        wrench_row(r, C.mu, C.fz, C.tm, gg, &hh);
        double gu = 0.0;
        for (int a = 0; a < 6; ++a) gu += gg[a] * u[a];
        const double sc = (r < 5) ? C.mg : C.tm;
        if (mu[r] * sc + (gu - hh) > 0.0) code |= (r < 5) ? (1 << r) : (1 << (8 + (r - 5)));
      }
      if (face_apex(code)) code = (code & ~31) | FACE_APEX;
      for (int a = 0; a < 3; ++a)
        if ((code >> (8 + a) & 1) && (code >> (11 + a) & 1)) code &= ~(1 << (11 + a));
    }
    C.faces[st * 2 + i] = code;
    uint64_t v = (uint64_t)(code + 1) * 0x9E3779B97F4A7C15ull ^ ((uint64_t)(e + 1) * 0xC2B2AE3D27D4EB4Full);
    v ^= v >> 29;
    v *= 0xBF58476D1CE4E5B9ull;
    hsh ^= v;
  }
  wsync();
  return wave_xor(hsh);
}

// Faces from slack: rows whose slack is below tol * row scale.
__device__ void faces_from_u(const Ctx& C, const double* u_src, double tol) {
  gsync();
  const int lane = threadIdx.x;
  for (int e = lane; e < C.N * 2; e += W64) {
    const int k = e >> 1, i = e & 1;
    const int st = k;
    int code = 0;
    if (C.contact[st * 2 + i]) {
      const double* u = u_src + st * NU + 6 * i;
      for (int r = 0; r < NROW; ++r) {
        double gg[6], hh;
        wrench_row(r, C.mu, C.fz, C.tm, gg, &hh);
        double gu = 0.0;
        for (int a = 0; a < 6; ++a) gu += gg[a] * u[a];
        const double sc = (r < 5) ? C.mg : C.tm;
        if ((hh - gu) / sc <= tol) code |= (r < 5) ? (1 << r) : (1 << (8 + (r - 5)));
      }
      if (face_apex(code)) code = (code & ~31) | FACE_APEX;
    }
    C.faces[st * 2 + i] = code;
  }
  wsync();
}

// One active-set pass: equality-constrained solve on the current faces,
// costates, multipliers and residuals.
__device__ double eq_pass(const Ctx& C, Sh& sh, double res[PINMPC_NRES]) {
  riccati(C, sh, Mode::EQ, true, nullptr);
  costates_grad(C, sh);
  const double kkt = multipliers_kkt(C, res);
  res[0] = dyn_residual(C);
  return fmax(kkt, res[0]);
}

// Interior-point fallback.  Rows scaled by mg (force rows) and tau_max
// (moment rows).  Leaves faces from z > s.
__device__ int ipm(const Ctx& C, Sh& sh, int maxit) {
  gsync();
  const int lane = threadIdx.x;
  const int N = C.N;
  // number of stance rows
  int mloc = 0;
  for (int e = lane; e < N * 2; e += W64)
    if (C.contact[(e >> 1) * 2 + (e & 1)]) mloc += NROW;
  const double m = wave_sum((double)mloc);
  if (m == 0.0) return 0;
  // initial point: the current ru (feasible ADMM point), its rollout in rx
  for (int e = lane; e < N * 2 * NROW; e += W64) {
    const int k = e / (2 * NROW), i = (e / NROW) & 1, r = e % NROW;
    const int st = k;
      const size_t rb = ((size_t)st * 2 + i) * NROW + r;
    if (!C.contact[st * 2 + i]) continue;
    double gg[6], hh;
    wrench_row(r, C.mu, C.fz, C.tm, gg, &hh);
    double gu = 0.0;
    for (int a = 0; a < 6; ++a) gu += gg[a] * C.ru[st * NU + 6 * i + a];
    const double sc = (r < 5) ? C.mg : C.tm;
    C.rs[rb] = fmax((hh - gu) / sc, 1.0);
    C.rz[rb] = 1.0;
  }
  wsync();
  double* rc = C.rdz;   // reuse: complementarity target, then dz
  int it = 0;
  for (; it < maxit; ++it) {
    // residuals rp and mu
    double smz = 0.0, rpn = 0.0;
    for (int e = lane; e < N * 2 * NROW; e += W64) {
      const int k = e / (2 * NROW), i = (e / NROW) & 1, r = e % NROW;
      const int st = k;
      const size_t rb = ((size_t)st * 2 + i) * NROW + r;
      if (!C.contact[st * 2 + i]) continue;
      double gg[6], hh;
      wrench_row(r, C.mu, C.fz, C.tm, gg, &hh);
      double gu = 0.0;
      for (int a = 0; a < 6; ++a) gu += gg[a] * C.ru[st * NU + 6 * i + a];
      const double sc = (r < 5) ? C.mg : C.tm;
      const double rp = (gu - hh) / sc + C.rs[rb];
      smz += C.rs[rb] * C.rz[rb];
      rpn = fmax(rpn, fabs(rp));
      rc[rb] = C.rs[rb] * C.rz[rb];     // affine (predictor) target
    }
    const double muv = wave_sum(smz) / m;
    rpn = wave_max(rpn);
    wsync();
    if (muv <= 1e-10 && rpn <= 1e-9) break;
    // predictor
    riccati(C, sh, Mode::NEWTON, true, rc);
    double amax_s = 1.0, amax_z = 1.0;
    for (int e = lane; e < N * 2 * NROW; e += W64) {
      const int k = e / (2 * NROW), i = (e / NROW) & 1, r = e % NROW;
      const int st = k;
      const size_t rb = ((size_t)st * 2 + i) * NROW + r;
      if (!C.contact[st * 2 + i]) continue;
      double gg[6], hh;
      wrench_row(r, C.mu, C.fz, C.tm, gg, &hh);
      double gu = 0.0, gdu = 0.0;
      for (int a = 0; a < 6; ++a) {
        gu += gg[a] * C.ru[st * NU + 6 * i + a];
        gdu += gg[a] * C.rdu[st * NU + 6 * i + a];
      }
      const double sc = (r < 5) ? C.mg : C.tm;
      const double s = C.rs[rb], z = C.rz[rb];
      const double rp = (gu - hh) / sc + s;
      const double ds = -rp - gdu / sc;
      const double dz = (-s * z - z * ds) / s;
      C.rds[rb] = ds;
      C.rmu[rb] = dz;     // affine dz kept in rmu scratch
      if (ds < 0) amax_s = fmin(amax_s, -s / ds);
      if (dz < 0) amax_z = fmin(amax_z, -z / dz);
    }
    const double aa = fmin(wave_min(amax_s), wave_min(amax_z));
    double sm = 0.0;
    for (int e = lane; e < N * 2 * NROW; e += W64) {
      const int k = e / (2 * NROW), i = (e / NROW) & 1;
      const int st = k;
      const size_t rb = ((size_t)st * 2 + i) * NROW + e % NROW;
      if (!C.contact[st * 2 + i]) continue;
      sm += (C.rs[rb] + aa * C.rds[rb]) * (C.rz[rb] + aa * C.rmu[rb]);
    }
    const double mu_aff = wave_sum(sm) / m;
    const double sigma = pow(mu_aff / muv, 3.0);
    wsync();
    for (int e = lane; e < N * 2 * NROW; e += W64) {
      const int k = e / (2 * NROW), i = (e / NROW) & 1;
      const int st = k;
      const size_t rb = ((size_t)st * 2 + i) * NROW + e % NROW;
      if (!C.contact[st * 2 + i]) continue;
      rc[rb] = C.rs[rb] * C.rz[rb] + C.rds[rb] * C.rmu[rb] - sigma * muv;
    }
    wsync();
    // corrector: same matrix, new right-hand side
    riccati(C, sh, Mode::NEWTON, false, rc);
    amax_s = 1.0;
    amax_z = 1.0;
    for (int e = lane; e < N * 2 * NROW; e += W64) {
      const int k = e / (2 * NROW), i = (e / NROW) & 1, r = e % NROW;
      const int st = k;
      const size_t rb = ((size_t)st * 2 + i) * NROW + r;
      if (!C.contact[st * 2 + i]) continue;
      double gg[6], hh;
      wrench_row(r, C.mu, C.fz, C.tm, gg, &hh);
      double gu = 0.0, gdu = 0.0;
      for (int a = 0; a < 6; ++a) {
        gu += gg[a] * C.ru[st * NU + 6 * i + a];
        gdu += gg[a] * C.rdu[st * NU + 6 * i + a];
      }
      const double sc = (r < 5) ? C.mg : C.tm;
      const double s = C.rs[rb], z = C.rz[rb];
      const double rp = (gu - hh) / sc + s;
      const double ds = -rp - gdu / sc;
      const double dz = (-rc[rb] - z * ds) / s;
      C.rds[rb] = ds;
      C.rmu[rb] = dz;
      if (ds < 0) amax_s = fmin(amax_s, -s / ds);
      if (dz < 0) amax_z = fmin(amax_z, -z / dz);
    }
    const double a = fmin(1.0, 0.99 * fmin(wave_min(amax_s), wave_min(amax_z)));
    wsync();
    for (int e = lane; e < N * 2 * NROW; e += W64) {
      const int k = e / (2 * NROW), i = (e / NROW) & 1;
      const int st = k;
      const size_t rb = ((size_t)st * 2 + i) * NROW + e % NROW;
      if (!C.contact[st * 2 + i]) continue;
      C.rs[rb] += a * C.rds[rb];
      C.rz[rb] += a * C.rmu[rb];
    }
    for (int e = lane; e < N * NU; e += W64) C.ru[e] += a * C.rdu[e];
    for (int e = lane; e < (N + 1) * NX; e += W64)
      C.rx[e] += a * C.rdx[e];
    wsync();
  }
  // faces from z > s (rows were updated by other lanes)
  gsync();
  for (int e = lane; e < N * 2; e += W64) {
    const int k = e >> 1, i = e & 1;
    const int st = k;
    int code = 0;
    if (C.contact[st * 2 + i]) {
      const size_t rb = (st * 2 + i) * NROW;
      for (int r = 0; r < NROW; ++r)
        if (C.rz[rb + r] > C.rs[rb + r]) code |= (r < 5) ? (1 << r) : (1 << (8 + (r - 5)));
      if (face_apex(code)) code = (code & ~31) | FACE_APEX;
      for (int a = 0; a < 3; ++a)
        if ((code >> (8 + a) & 1) && (code >> (11 + a) & 1)) code &= ~(1 << (11 + a));
    }
    C.faces[st * 2 + i] = code;
  }
  wsync();
  return it;
}

// Active-set loop; returns true if certified.  passes accumulates.
__device__ bool active_set_loop(const Ctx& C, Sh& sh, int maxp, double tol, int* passes,
                                double res[PINMPC_NRES], double* kkt_out) {
  uint64_t hist[8];
  for (int i = 0; i < 8; ++i) hist[i] = 0;
  int nh = 0;
  for (int it = 0; it < maxp; ++it) {
    const double kkt = eq_pass(C, sh, res);
    ++*passes;
    *kkt_out = kkt;
    if (kkt <= tol) return true;
    const uint64_t h = pdas_update(C);
    bool seen = false;
    for (int i = 0; i < 8; ++i) seen |= (hist[i] == h) && (i < nh || nh >= 8);
    if (seen) return false;
    hist[nh & 7] = h;
    ++nh;
  }
  return false;
}

__device__ void rollout_ru(const Ctx& C, Sh& sh) {
  gsync();
  // x = rollout of ru from x0, in FP64, into rx
  const int lane = threadIdx.x;
  if (lane < NX) sh.xv[lane] = (double)C.x0[lane];
  wsync();
  if (lane < NX) C.rx[lane] = sh.xv[lane];
  for (int k = 0; k < C.N; ++k) {
    if (lane < NX) {
      double acc = C.e ? (double)C.e[k * NX + lane] : 0.0;
      for (int l = 0; l < NX; ++l) acc += (double)C.A[k * NX * NX + lane * NX + l] * sh.xv[l];
      for (int l = 0; l < NU; ++l) acc += (double)C.B[k * NX * NU + lane * NU + l] * C.ru[k * NU + l];
      sh.xn[lane] = acc;
    }
    wsync();
    if (lane < NX) {
      sh.xv[lane] = sh.xn[lane];
      C.rx[(k + 1) * NX + lane] = sh.xn[lane];
    }
    wsync();
  }
}

// The ADMM's input iterate, unscaled, into ru (swing inputs exactly 0).
__device__ void admm_point(const Ctx& C, const float* zsrc, const float* sf, float tsc) {
  gsync();
  const int lane = threadIdx.x;
  for (int e = lane; e < C.N * NU; e += W64) {
    const int k = e / NU, j = e % NU;
    const double sc = (j % 6 < 3) ? (double)sf[k] : (double)tsc;
    double v = (double)zsrc[((size_t)k * NSTATE) * NL + NX + j] * sc;
    if (!C.contact[k * 2 + j / 6]) v = 0.0;
    C.ru[k * NU + j] = v;
  }
  wsync();
}

__global__ void __launch_bounds__(64) refine_kernel(Problem p, Workspace ws, float* out_u,
                                                    float* out_x, float* out_res,
                                                    int32_t* out_iters, int32_t* out_status,
                                                    int admm_iters, int accel, int refine,
                                                    int pass_a, int ipm_max, int pass_c,
                                                    double tol) {
  __shared__ Sh sh;
  // the problem context lives in LDS: its pointers are loaded where they are
  // used instead of being held in registers across the whole kernel
  __shared__ Ctx C;
  const int lane = threadIdx.x;
  if (lane == 0) {
  C.b = blockIdx.x;
  C.n = p.n_max;
  C.N = horizon(p, C.b);
  const size_t s0 = (size_t)C.b * C.n;
  C.mu = p.mu[C.b];
  C.fz = p.fz_max[C.b];
  C.tm = p.tau_max[C.b];
  C.mg = weight_of(p, C.b);
  C.Q = sh.Qd;
  C.R = sh.Rd;
  C.A = p.A + s0 * NX * NX;
  C.B = p.B + s0 * NX * NU;
  C.e = p.e ? p.e + s0 * NX : nullptr;
  C.x_ref = p.x_ref + s0 * NX;
  C.u_ref = p.u_ref ? p.u_ref + s0 * NU : nullptr;
  C.x0 = p.x0 + (size_t)C.b * NX;
  C.contact = p.contact + s0 * 2;
  {
    const int n = C.n;
    double* blk = ws.rblk + (size_t)C.b * refine_block_doubles(n);
    C.rK = blk;                       blk += (size_t)n * NU * NX;
    C.rkap = blk;                     blk += (size_t)n * NU;
    C.rL = blk;                       blk += (size_t)n * NU * NU;
    C.rHwx = blk;                     blk += (size_t)n * NU * NX;
    C.ru = blk;                       blk += (size_t)n * NU;
    C.rx = blk;                       blk += (size_t)(n + 1) * NX;
    C.rlam = blk;                     blk += (size_t)n * NX;
    C.rg = blk;                       blk += (size_t)n * NU;
    C.rmu = blk;                      blk += (size_t)n * 2 * NROW;
    C.rs = blk;                       blk += (size_t)n * 2 * NROW;
    C.rz = blk;                       blk += (size_t)n * 2 * NROW;
    C.rds = blk;                      blk += (size_t)n * 2 * NROW;
    C.rdz = blk;                      blk += (size_t)n * 2 * NROW;
    C.rdu = blk;                      blk += (size_t)n * NU;
    C.rdx = blk;                      blk += (size_t)(n + 1) * NX;
    C.ftab = blk;                     blk += (size_t)n * 2 * FT;
    C.wrow = blk;                     blk += (size_t)n * 2 * NROW;
    C.crow = blk;
    C.faces = ws.faces + s0 * 2;
  }
  }
  if (lane < NX) sh.Qd[lane] = p.Q[(size_t)blockIdx.x * NX + lane];
  if (lane < NU) sh.Rd[lane] = p.R[(size_t)blockIdx.x * NU + lane];
  wsync();
  const size_t s0 = (size_t)blockIdx.x * p.n_max;
  const int N = C.N;

  // input checks: bounds, then finiteness of this problem's data
  const int Nraw = horizon_raw(p, C.b);
  int bad = !(C.mu >= 0.0) || !(C.fz >= 0.0) || !(C.tm >= 0.0) || !(C.mg > 0.0) ||
            Nraw < 1 || Nraw > C.n;
  for (int j = 0; j < NX; ++j) bad |= !(C.Q[j] > 0.0);
  for (int j = 0; j < NU; ++j) bad |= !(C.R[j] > 0.0);
  int nonfinite = 0;
  if (!bad) {
    for (int e = lane; e < N * NX * NX; e += W64) nonfinite |= !isfinite(C.A[e]);
    for (int e = lane; e < N * NX * NU; e += W64) nonfinite |= !isfinite(C.B[e]);
    for (int e = lane; e < N * NX; e += W64) {
      nonfinite |= !isfinite(C.x_ref[e]);
      if (C.e) nonfinite |= !isfinite(C.e[e]);
    }
    if (lane < NX) nonfinite |= !isfinite(C.x0[lane]);
  }
  nonfinite = wave_max((double)nonfinite) > 0.0;
  const size_t ux = (size_t)C.b * C.n * NU, xx = (size_t)C.b * (C.n + 1) * NX;
  if (bad || nonfinite) {
    for (int e = lane; e < C.n * NU; e += W64) out_u[ux + e] = 0.f;
    for (int e = lane; e < (C.n + 1) * NX; e += W64) out_x[xx + e] = 0.f;
    if (lane == 0) {
      if (out_status) out_status[C.b] = bad ? PINMPC_ST_BADINPUT : PINMPC_ST_NONFINITE;
      if (out_iters) out_iters[C.b] = 0;
    }
    if (out_res && lane < PINMPC_NRES) out_res[(size_t)C.b * PINMPC_NRES + lane] = __builtin_nanf("");
    return;
  }

  const float* zsrc = (accel ? ws.cur : ws.hat) + s0 * NSTATE * NL;
  const float* sf = ws.sf + s0;
  const float tsc = ws.tsc[C.b];
  admm_point(C, zsrc, sf, tsc);

  double res[PINMPC_NRES] = {0, 0, 0, 0, 0};
  double kkt = 1e300;
  int passes = 0;
  bool ok = false;
  if (refine) {
    faces_from_u(C, C.ru, 1e-5);
    ok = active_set_loop(C, sh, pass_a, tol, &passes, res, &kkt);
    if (!ok && ipm_max > 0) {
      // interior point from the ADMM point (ru was overwritten by the passes)
      admm_point(C, zsrc, sf, tsc);
      rollout_ru(C, sh);
      const int its = ipm(C, sh, ipm_max);
      passes += its;
      ok = active_set_loop(C, sh, pass_c, tol, &passes, res, &kkt);
    }
  } else {
    // the ADMM point as it is: rollout, faces from slack, residuals
    faces_from_u(C, C.ru, 1e-5);
    rollout_ru(C, sh);
    costates_grad(C, sh);
    kkt = multipliers_kkt(C, res);
    res[0] = dyn_residual(C);
  }

  // outputs
  gsync();
  for (int e = lane; e < C.n * NU; e += W64)
    out_u[ux + e] = (e < N * NU) ? (float)C.ru[e] : 0.f;
  for (int e = lane; e < (C.n + 1) * NX; e += W64)
    out_x[xx + e] = (e < (N + 1) * NX) ? (float)C.rx[e] : 0.f;
  if (lane == 0) {
    if (out_status)
      out_status[C.b] = refine ? (ok ? PINMPC_ST_OK : PINMPC_ST_UNPOLISHED) : PINMPC_ST_MAXITER;
    if (out_iters) out_iters[C.b] = admm_iters + passes;
  }
  if (out_res) {
    for (int i = 0; i < PINMPC_NRES; ++i)
      if (lane == i) out_res[(size_t)C.b * PINMPC_NRES + i] = (float)res[i];
  }
}

}  // namespace

hipError_t launch_refine(const Problem& p, const Workspace& w, const pinmpc_settings& s,
                         const pinmpc_out& out, hipStream_t st) {
  if (p.batch == 0) return hipSuccess;
  hipLaunchKernelGGL(refine_kernel, dim3(p.batch), dim3(64), 0, st, p, w, out.u, out.x, out.res,
                     out.iters, out.status, s.iters, s.accel, s.refine, s.refine_passes,
                     s.ipm_iters, s.polish_passes, s.kkt_tol);
  return hipGetLastError();
}

}  // namespace pinmpc
