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

// Pointers with their address space spelled out: the context lives in LDS,
// so the compiler cannot infer where its pointers point, and generic (flat)
// accesses would make every wait on one load a wait on all memory in flight.
#define GMEM __attribute__((address_space(1)))
#define LMEM __attribute__((address_space(3)))
typedef const GMEM float* gcf;
typedef const GMEM double* gcd;
typedef GMEM double* gd;

// One problem's view: its inputs and its FP64 scratch block, all as
// pointers to the problem's own first stage, so stage k is plain k.
struct Ctx {
  int b, N, n;
  double mu, fz, tm, mg;
  const LMEM double* Q;   // LDS copies of the diagonal weights
  const LMEM double* R;
  gcf A, B, e, x_ref, u_ref, x0;
  const GMEM uint8_t* contact;
  gd rT, rK, rL, rHwx, rS;   // per-stage compact blocks (TS_T, TS_K, ... doubles)
  gd rkap, ru, rx, rlam, rg, rmu, rs, rz, rds, rdz, rdu, rdx;
  gd rPV, rGV;   // long horizons: the stage buffers of the rollout and costates
  GMEM int32_t* faces;
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
// With the associative scan of the backward recursion a problem's workgroup
// holds several waves; the first runs the refinement and the others join it
// only at the scan's own barriers.  There, the hand-off between lanes of the
// first wave needs the fence alone (the waves of a workgroup share the CU's
// caches), never the workgroup barrier.
__device__ inline void gsync() {
  if (blockDim.x == W64) {
    __syncthreads();
  } else {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
  }
}
// lane within the wave (the workgroup may hold several waves)
__device__ inline int lane_id() { return (int)(threadIdx.x & 63); }

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
#pragma unroll 1
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

// --------------------------------------------------------------- LDS state

// Hand-off buffers of the stage recursion; everything else of a stage lives
// in registers as 16 x 16 tiles.
constexpr int GS = NU + NX + 2;   // row stride of the Gauss-Jordan hand-off
struct ShR {
  double G[NU * GS];     // [H | Hwx | hw] of the stage, row-major
  double KK[NU * 16];    // [K | 0 | kap]: gains, feedforward in column 13
  double HI[NU * 16];    // H^{-1} (Newton steps, chunk summaries)
  double ST[16 * 17];    // S of the stage, for its transpose
};
struct Sh {
  // the Riccati recursion's hand-off buffers and the costate recursion's
  // stage vectors share storage: the two never run at the same time
  union {
    ShR r;
    struct {
      double PV[PINMPC_NMAX * 16];   // Q (x_{k+1} - r_k), then p_{k+1}
      double GV[PINMPC_NMAX * 16];   // R (u_k - u_ref_k), then g_k
    } c;
  };
  double xv[NX], xn[NX];
  double Qd[NX], Rd[NU]; // diagonal weights of the problem
};

// The per-stage 16-wide vectors of the rollout and the costate chain: in LDS
// up to PINMPC_NMAX stages; for longer horizons (LONG) in the problem's scratch
// block, where a hand-off between lanes needs the barrier with its memory fence
// instead of the wave's LDS ordering.
template <bool LONG>
struct StageBufs;
template <>
struct StageBufs<false> {
  double* PV;
  double* GV;
  __device__ StageBufs(Sh& sh, const Ctx&) : PV(sh.c.PV), GV(sh.c.GV) {}
};
template <>
struct StageBufs<true> {
  gd PV;
  gd GV;
  __device__ StageBufs(Sh&, const Ctx& C) : PV(C.rPV), GV(C.rGV) {}
};
template <bool LONG>
__device__ inline void bufsync() {
  if constexpr (LONG) gsync();
  else wsync();
}

// ------------------------------------------------------------ 16 x 16 tiles
//
// The stage recursion works on 16 x 16 FP64 tiles (13 states, 12 inputs, zero
// padded) held in registers in the result layout of the FP64 matrix-core
// product (16 x 16 x 4 per instruction): lane l = 16 g + j holds items
// q = 0..3, item q being entry (4 q + g, j).  The same layout is the right
// operand of the product chunk by chunk, and read as the left operand it is
// the transposed tile.  So for tiles U, V in registers mmT(U, V) = U^T V takes
// four instructions and leaves a tile again: products chain with no data
// movement.  Vectors ride in column VC of a tile (lanes 13, 29, 45, 61).

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int VC = 13;

__device__ inline d4 zero4() {
  d4 z = {0.0, 0.0, 0.0, 0.0};
  return z;
}
__device__ inline int tg() { return lane_id() >> 4; }
__device__ inline int tj() { return lane_id() & 15; }

// U^T V + acc, contracting over the first 4 NQ rows (NQ = 3: the input rows).
template <int NQ>
__device__ inline d4 mmT(d4 u, d4 v, d4 acc) {
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(u[q], v[q], acc, 0, 0, 0);
  return acc;
}

// Column-VC vector of a tile to / from memory (len entries).
__device__ inline void vec_store(gd v, int len, d4 t) {
  if (tj() == VC) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (4 * q + tg() < len) v[4 * q + tg()] = t[q];
  }
}
__device__ inline d4 sel(bool c, d4 a) { return c ? a : zero4(); }

// Stage blocks in memory hold only the entries a tile can have nonzero (the
// layouts are listed with refine_block_doubles).  A map packs, for each of a
// lane's four tile items, the item's offset in the block (in doubles, 8 bits
// per item) or 255 for an item the block does not hold.  Blocks are read and
// written with buffer instructions whose range is the block: an item mapped
// to 255 lies past the end (255 doubles exceed every block), so its load
// returns zero and its store is dropped by the hardware's range check.  A
// fetch issued a stage ahead thus needs no masking and stores need no
// branches.
constexpr uint32_t NOT_HELD = 255;
static_assert(TS_T < 255 && TS_K < 255 && TS_L < 255 && TS_H < 255 && TS_S < 255,
              "a stage block must end before the out-of-range offset");
__device__ inline uint32_t pack_map(const int o[4]) {
  uint32_t m = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) m |= (uint32_t)o[q] << (8 * q);
  return m;
}
// rows x cols, row-major
__device__ inline uint32_t map_rect(int rows, int cols) {
  int o[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = 4 * q + tg(), c = tj();
    o[q] = (r < rows && c < cols) ? r * cols + c : (int)NOT_HELD;
  }
  return pack_map(o);
}
// stage input block: the two contacts' 6 x 6 diagonal blocks and offsets
__device__ inline uint32_t map_T() {
  int o[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = 4 * q + tg(), c = tj();
    const bool blk = r < NU && c < NU && (r / 6) == (c / 6);
    const bool off = r < NU && c == VC;
    o[q] = blk ? (r / 6) * 42 + (r % 6) * 6 + (c % 6)
               : (off ? (r / 6) * 42 + 36 + (r % 6) : (int)NOT_HELD);
  }
  return pack_map(o);
}
// value function: S symmetric (13 x 13, lower triangle), s in column VC;
// `store` selects the lower triangle only, a load reads both triangles
__device__ inline uint32_t map_S(bool store) {
  int o[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = 4 * q + tg(), c = tj();
    const int hi = r > c ? r : c, lo = r > c ? c : r;
    const bool sym = r < NX && c < NX && (!store || c <= r);
    const bool vec = r < NX && c == VC;
    o[q] = sym ? hi * (hi + 1) / 2 + lo : (vec ? NX * (NX + 1) / 2 + r : (int)NOT_HELD);
  }
  return pack_map(o);
}
typedef unsigned int u2 __attribute__((ext_vector_type(2)));
// buffer resource over one stage block of `doubles` entries (raw buffer:
// stride 0, 32-bit data format, range checked against the block's bytes)
__device__ inline __amdgpu_buffer_rsrc_t block_rsrc(gcd base, int doubles) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, 0, doubles * 8, 0x00020000);
}
// Item q's byte offset, kept in a vector register: an offset the compiler
// could prove constant would otherwise move into the instruction's immediate
// field, and the range check is meant to see every offset the same way.
__device__ inline int map_offset(uint32_t map, int q) {
  int off = (int)(((map >> (8 * q)) & 255) * 8);
  asm volatile("" : "+v"(off));
  return off;
}
// (Element values move through memcpy: a bit cast applied directly to a
// vector element has been seen to read element 0 for every element.)
__device__ inline d4 ld_map(gcd base, int doubles, uint32_t map) {
  const __amdgpu_buffer_rsrc_t r = block_rsrc(base, doubles);
  d4 t;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const u2 w = __builtin_amdgcn_raw_buffer_load_b64(r, map_offset(map, q), 0, 0);
    double v;
    __builtin_memcpy(&v, &w, 8);
    t[q] = v;
  }
  return t;
}
__device__ inline void st_map(gd base, int doubles, uint32_t map, d4 t) {
  const __amdgpu_buffer_rsrc_t r = block_rsrc(base, doubles);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double v = t[q];
    u2 w;
    __builtin_memcpy(&w, &v, 8);
    __builtin_amdgcn_raw_buffer_store_b64(w, r, map_offset(map, q), 0, 0);
  }
}

// Stage input blocks, written in parallel over (stage, contact): each lane
// computes one contact's 6 x 6 diagonal block and its six offsets (column VC
// of the tile) in registers and stores them, whole, into the stage's block
// (zero for a swing contact).
//   equality passes: the face projector P (block diagonal) and the face
//                    offset c of the contact;
//   Newton steps:    the input Hessian R + G^T diag(z/s) G and the linear term
//                    R (u - u_ref) + G^T c_rows of a stance contact (zero
//                    for a swing contact).
// Interior-point rows are scaled by sc (mg force rows, tau_max moment rows):
// row weight z / (s sc^2), linear coefficient (z + (-rc + z rp) / s) / sc with
// rp = (g u - h) / sc + s.
__device__ void build_tiles(const Ctx& C, bool newton, gcd rcvec, int kn) {
  const int lane = lane_id();
  for (int e = lane; e < kn * 2; e += W64) {
    const int k = e >> 1, i = e & 1;
    gd base = C.rT + (size_t)k * TS_T + i * 42;
    double P6[6][6], c6[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      c6[a] = 0.0;
#pragma unroll
      for (int b = 0; b < 6; ++b) P6[a][b] = 0.0;
    }
    if (C.contact[k * 2 + i]) {
      if (!newton) {
        face_affine(C.faces[k * 2 + i], C.mu, C.fz, C.tm, P6, c6);
      } else {
        double u[6];
#pragma unroll
        for (int a = 0; a < 6; ++a) {
          const int jj = 6 * i + a;
          u[a] = C.ru[k * NU + jj];
          const double ur = C.u_ref ? (double)C.u_ref[k * NU + jj] : 0.0;
          P6[a][a] = C.R[jj];
          c6[a] = C.R[jj] * (u[a] - ur);
        }
        const size_t rb = (size_t)e * NROW;
#pragma unroll
        for (int row = 0; row < NROW; ++row) {
          double gr[6], h;
          wrench_row(row, C.mu, C.fz, C.tm, gr, &h);
          const double sc = (row < 5) ? C.mg : C.tm;
          double gu = 0.0;
#pragma unroll
          for (int a = 0; a < 6; ++a) gu += gr[a] * u[a];
          const double s = C.rs[rb + row], z = C.rz[rb + row];
          const double rp = (gu - h) / sc + s;
          const double w = z / s / (sc * sc);
          const double cr = (z + (-rcvec[rb + row] + z * rp) / s) / sc;
#pragma unroll
          for (int a = 0; a < 6; ++a) {
            c6[a] += gr[a] * cr;
#pragma unroll
            for (int b = 0; b < 6; ++b) P6[a][b] += w * gr[a] * gr[b];
          }
        }
      }
    }
#pragma unroll
    for (int a = 0; a < 6; ++a) {
#pragma unroll
      for (int b = 0; b < 6; ++b) base[a * 6 + b] = P6[a][b];
      base[36 + a] = c6[a];
    }
  }
}

// ------------------------------------------------------ Riccati recursion
//
// Solves   min sum_k 1/2 x_{k+1}^T Q x_{k+1} + q_k^T x_{k+1}
//                    + 1/2 u_k^T R'_k u_k + rho_k^T u_k
//          s.t. x_{k+1} = A_k x_k + B_k u_k + e_k,  u_k = c_k + P_k w_k
// (P_k an orthogonal projector) by the backward recursion on the value
// function V(x) = 1/2 x^T S x + s^T x and the forward rollout.
//   EQ:     the equality-constrained tracking problem of the faces
//           (q = -Q r, rho = -R u_ref, R' = R, e from the data);
//   NEWTON: the interior-point Newton step, x_0 = 0, e = 0,
//           q = Q (x_{k+1} - r), R' = R + G^T diag(z/s) G,
//           rho from the stage tile, P = stance mask, c = 0.
// Per stage, with W = S + Q, Bp = B P and d = B c + e:
//   H = P R' P + Bp^T W Bp + (I - P),  Hwx = Bp^T W A,
//   hw = P (R' c + rho) + Bp^T (W d + q + s),
//   K = -H^{-1} Hwx, kap = -H^{-1} hw,
//   S <- A^T W A + Hwx^T K,  s <- A^T (W d + q + s) + Hwx^T kap.
// With factor = false only the linear part is recomputed from the stored
// H^{-1}, Hwx and K (second right-hand side of the same Newton matrix).
// EQ keeps each stage's value function [S_k | s_k] (symmetrised, as used);
// stage k's factors depend on the faces of stages k..N-1 only, so a pass
// whose faces differ from the previous pass's only before stage ktop
// rebuilds the tiles and reruns the backward recursion for stages
// 0..ktop-1 only, starting from the kept [S_ktop | s_ktop]; the result is
// bitwise that of the whole recursion.

enum class Mode { EQ, NEWTON };

// Raw stage data.  The stage loops fetch the next stage's data a whole stage
// ahead; the fetch only gathers (addresses clamped into the stage's arrays)
// and the conversion and masking happen when the stage is used.  Before the
// next fetch and the deferred stores are issued, everything the stage uses is
// pinned in registers, so no wait on memory falls inside a stage's compute
// (loads and stores share one counter here: waiting for any access would
// otherwise mean waiting for all of them).
__device__ inline int clampi(int v, int hi) { return v < hi ? v : hi; }
__device__ inline void gather(gcf M, bool transposed, int rows, int cols, float m[4]) {
  const int g = tg(), j = tj();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = 4 * q + g;
    m[q] = transposed ? M[clampi(j, rows - 1) * cols + clampi(r, cols - 1)]
                      : M[clampi(r, rows - 1) * cols + clampi(j, cols - 1)];
  }
}
__device__ inline void gatherv(gcf v, int len, float m[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) m[q] = v[clampi(4 * q + tg(), len - 1)];
}
__device__ inline d4 cook(const float m[4], bool transposed, int rows, int cols) {
  const int g = tg(), j = tj();
  d4 t;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = 4 * q + g;
    const bool ok = transposed ? (j < rows && r < cols) : (r < rows && j < cols);
    t[q] = ok ? (double)m[q] : 0.0;
  }
  return t;
}
__device__ inline void pin(const d4& t) {
  asm volatile("" ::"v"(t[0]), "v"(t[1]), "v"(t[2]), "v"(t[3]));
}
__device__ inline void pin(double t) { asm volatile("" ::"v"(t)); }
__device__ inline void pin_memory() { asm volatile("" ::: "memory"); }
// A pointer read from the LDS context, made wave-uniform (scalar registers):
// the stage loops then neither re-read the context after their LDS stores
// nor hold its pointers in vector registers.
template <class T>
__device__ inline T uni(T p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return (T)(((uint64_t)hi << 32) | lo);
}

// Stance mask tile (identity on the inputs of stance contacts).
__device__ inline d4 mask_tile(int stance) {
  const int g = tg(), j = tj();
  const double m = (j < NU && stance) ? 1.0 : 0.0;
  d4 p;
#pragma unroll
  for (int q = 0; q < 4; ++q) p[q] = (4 * q + g == j) ? m : 0.0;
  return p;
}

struct BackRaw {
  float a[4], bt[4], xr[4], ev[4], ur[4];
  double xn[4];
  d4 T, HI, HX;
  int ct;
  int c0, c1, f0, f1;   // the stage's contact flags and face codes (uniform)
};

// Inputs of a stage that the projector P_k removes exactly (P_k's column is
// zero): every input of a swing contact; on an equality pass also the force of
// an apex face and each moment component fixed at its bound.  For those, the
// stage system [H | Hwx | hw] has exactly e_j as row and column j.
__device__ inline uint32_t null_inputs(int c0, int c1, int f0, int f1, bool newton) {
  uint32_t m = 0;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int c = i ? c1 : c0, f = i ? f1 : f0;
    if (!c) {
      m |= 0x3Fu << (6 * i);
    } else if (!newton) {
      if ((f & 31) == FACE_APEX) m |= 7u << (6 * i);
#pragma unroll
      for (int a = 0; a < 3; ++a)
        if (((f >> (8 + a)) & 1) || ((f >> (11 + a)) & 1)) m |= 1u << (6 * i + 3 + a);
    }
  }
  return m;
}

// s + sum_r (v of lane r of this 16-lane row) * a[r], r = 0..12, over four
// interleaved accumulators: the DPP row broadcast of v rides in each fused
// multiply-add.  The leading two wait states separate the block's DPP reads
// of v from a vector write of v just before it.
__device__ inline double dot_row_bcast13(double v, const double (&a)[13], double s) {
  double s1 = 0.0, s2 = 0.0, s3 = 0.0;
#define PINMPC_DOT(acc, r, ai) \
  "v_fmac_f64_dpp %" #acc ", %4, %" #ai " row_newbcast:" #r " row_mask:0xf bank_mask:0xf bound_ctrl:1\n"
  asm volatile("s_nop 1\n"
               PINMPC_DOT(0, 0, 5) PINMPC_DOT(1, 1, 6) PINMPC_DOT(2, 2, 7) PINMPC_DOT(3, 3, 8)
               PINMPC_DOT(0, 4, 9) PINMPC_DOT(1, 5, 10) PINMPC_DOT(2, 6, 11) PINMPC_DOT(3, 7, 12)
               PINMPC_DOT(0, 8, 13) PINMPC_DOT(1, 9, 14) PINMPC_DOT(2, 10, 15)
               PINMPC_DOT(3, 11, 16) PINMPC_DOT(0, 12, 17)
               : "+v"(s), "+v"(s1), "+v"(s2), "+v"(s3)
               : "v"(v), "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3]), "v"(a[4]), "v"(a[5]),
                 "v"(a[6]), "v"(a[7]), "v"(a[8]), "v"(a[9]), "v"(a[10]), "v"(a[11]),
                 "v"(a[12]));
#undef PINMPC_DOT
  return (s + s1) + (s2 + s3);
}

// s + sum_r (v of lane r of this 16-lane row) * a[r], r = 0..11, likewise.
__device__ inline double dot_row_bcast12(double v, const double (&a)[12], double s) {
  double s1 = 0.0, s2 = 0.0, s3 = 0.0;
#define PINMPC_DOT(acc, r, ai) \
  "v_fmac_f64_dpp %" #acc ", %4, %" #ai " row_newbcast:" #r " row_mask:0xf bank_mask:0xf bound_ctrl:1\n"
  asm volatile("s_nop 1\n"
               PINMPC_DOT(0, 0, 5) PINMPC_DOT(1, 1, 6) PINMPC_DOT(2, 2, 7) PINMPC_DOT(3, 3, 8)
               PINMPC_DOT(0, 4, 9) PINMPC_DOT(1, 5, 10) PINMPC_DOT(2, 6, 11) PINMPC_DOT(3, 7, 12)
               PINMPC_DOT(0, 8, 13) PINMPC_DOT(1, 9, 14) PINMPC_DOT(2, 10, 15)
               PINMPC_DOT(3, 11, 16)
               : "+v"(s), "+v"(s1), "+v"(s2), "+v"(s3)
               : "v"(v), "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3]), "v"(a[4]), "v"(a[5]),
                 "v"(a[6]), "v"(a[7]), "v"(a[8]), "v"(a[9]), "v"(a[10]), "v"(a[11]));
#undef PINMPC_DOT
  return (s + s1) + (s2 + s3);
}

// Backward recursion over stages k_hi - 1 down to k_lo from the value
// function Ss of x_{k_hi} (S in columns 0..12, s in VC); returns the value
// function of x_{k_lo}.  It stores each stage's gains and feedforward (and,
// for equality passes, its value function; for Newton steps H^-1 and Hwx).
// ELEM: the chunk summary of the associative scan instead (see below): the
// recursion starts from a zero value at x_{k_hi}, stores nothing and also
// composes the closed-loop affine map TE (transposed, offset in row 13,
// (13, 13) = 1) and the reachability term CE of the chunk.
template <Mode mode, bool factor, bool LONG, bool ELEM>
__device__ __attribute__((always_inline)) inline d4 backward(const Ctx& C, ShR& sr, int k_lo,
                                                             int k_hi, d4 Ss, d4* TEo, d4* CEo) {
  static_assert(!ELEM || factor, "a chunk summary factors every stage");
  const int lane = lane_id(), g = tg(), j = tj();
  constexpr bool newton = (mode == Mode::NEWTON);
  const gcf pA = uni(C.A), pB = uni(C.B), pxr = uni(C.x_ref), pe = uni(C.e), pur = uni(C.u_ref);
  const GMEM uint8_t* pct = uni(C.contact);
  const GMEM int32_t* pfc = uni(C.faces);
  const gd prT = uni(C.rT), prK = uni(C.rK), prL = uni(C.rL), prH = uni(C.rHwx), prS = uni(C.rS);
  const gd prkap = uni(C.rkap), prx = uni(C.rx), pru = uni(C.ru), prdx = uni(C.rdx),
           prdu = uni(C.rdu);
  // the diagonal weights where this lane uses them
  const double Qj = C.Q[clampi(j, NX - 1)];
  d4 Qr, Rr;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    Qr[q] = C.Q[clampi(4 * q + g, NX - 1)];
    Rr[q] = C.R[clampi(4 * q + g, NU - 1)];
  }
  // maps of the stage blocks this variant moves
  const uint32_t mT = map_T();
  const uint32_t mS = map_S(true);
  const uint32_t mL = map_rect(NU, NU), mH = map_rect(NU, NX);
  auto fetch = [&](int k, BackRaw& s) {
    gather(pA + (size_t)k * NX * NX, false, NX, NX, s.a);
    gather(pB + (size_t)k * NX * NU, true, NX, NU, s.bt);
    gatherv(pxr + (size_t)k * NX, NX, s.xr);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      s.ev[q] = 0.f;
      s.ur[q] = 0.f;
      s.xn[q] = 0.0;
    }
    if (!newton && pe) gatherv(pe + (size_t)k * NX, NX, s.ev);
    if (!newton && pur) gatherv(pur + (size_t)k * NU, NU, s.ur);
    if (newton) {
#pragma unroll
      for (int q = 0; q < 4; ++q) s.xn[q] = prx[(size_t)(k + 1) * NX + clampi(4 * q + g, NX - 1)];
    }
    s.T = ld_map(prT + (size_t)k * TS_T, TS_T, mT);
    if (newton && !factor) {
      s.HI = ld_map(prL + (size_t)k * TS_L, TS_L, mL);
      s.HX = ld_map(prH + (size_t)k * TS_H, TS_H, mH);
    } else {
      s.HI = s.HX = zero4();
    }
    s.ct = newton ? (int)pct[k * 2 + (j < NU ? j / 6 : 0)] : 0;
    s.c0 = __builtin_amdgcn_readfirstlane((int)pct[k * 2]);
    s.c1 = __builtin_amdgcn_readfirstlane((int)pct[k * 2 + 1]);
    s.f0 = newton ? 0 : __builtin_amdgcn_readfirstlane(pfc[k * 2]);
    s.f1 = newton ? 0 : __builtin_amdgcn_readfirstlane(pfc[k * 2 + 1]);
  };

  BackRaw raw;
  fetch(k_hi > k_lo ? k_hi - 1 : k_lo, raw);
  d4 TE = zero4(), CE = zero4();
  if constexpr (ELEM) {
#pragma unroll
    for (int q = 0; q < 4; ++q) TE[q] = (4 * q + g == j && j <= VC) ? 1.0 : 0.0;
  }
  for (int k = k_hi - 1; k >= k_lo; --k) {
    // this stage's data
    const d4 At = cook(raw.a, false, NX, NX);
    const d4 BT = cook(raw.bt, true, NX, NU);
    const d4 T = raw.T, HIs = raw.HI, HXs = raw.HX;
    d4 om, ev, ur;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = 4 * q + g;
      const bool vr = (j == VC && r < NX);
      const double xr = (double)raw.xr[q];
      om[q] = vr ? (newton ? Qr[q] * (raw.xn[q] - xr) : -Qr[q] * xr) : 0.0;
      ev[q] = vr ? (double)raw.ev[q] : 0.0;
      ur[q] = (j == VC && r < NU) ? (double)raw.ur[q] : 0.0;
    }
    if (ELEM && k == k_hi - 1) {
      // a zero value at x_{k_hi}: S = -Q and s = -q make W = S + Q and
      // q + s vanish at the chunk's last stage
#pragma unroll
      for (int q = 0; q < 4; ++q)
        Ss[q] = (j < NX && 4 * q + g == j) ? -Qj : ((j == VC) ? -om[q] : 0.0);
    }
    const d4 Pt = newton ? mask_tile(raw.ct) : sel(j < NU, T);
    const uint32_t unit = null_inputs(raw.c0, raw.c1, raw.f0, raw.f1, newton);
    pin(At); pin(BT); pin(T); pin(om); pin(ev); pin(ur); pin(Pt);
    if (newton && !factor) { pin(HIs); pin(HXs); }
    pin_memory();
    if (k > k_lo) fetch(k - 1, raw);

    // [Bp | 0 | d] = B [P | 0 | c] + [0 | 0 | e]
    const d4 yc = (!newton && j == VC) ? T : Pt;
    d4 D1 = mmT<3>(BT, yc, ev);
    d4 PRP = zero4();
    if (!newton && factor) {
      d4 RP;
#pragma unroll
      for (int q = 0; q < 4; ++q) RP[q] = (j < NU && 4 * q + g < NU) ? Rr[q] * T[q] : 0.0;
      const d4 Py = (j < NU) ? T : sel(j == VC, T - ur);
      PRP = mmT<3>(RP, Py, zero4());
    }
    const d4 Bp = sel(j < NU, D1);
    d4 Sn;
    if (factor) {
      d4 Wt;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        Wt[q] = (j < NX) ? Ss[q] + ((4 * q + g == j) ? Qj : 0.0) : 0.0;
      const d4 yA = (j < NX) ? At : sel(j == VC, D1);
      d4 D2 = mmT<4>(Wt, yA, zero4());      // [W A | W d]
      if (j == VC) D2 += om + Ss;            // [W A | W d + q + s]
      const d4 D3 = mmT<4>(Wt, Bp, zero4()); // W Bp
      d4 D4 = mmT<4>(Bp, D3, zero4());       // Bp^T W Bp
      const d4 D5 = mmT<4>(Bp, D2, zero4()); // [Hwx | Bp^T (W d + q + s)]
      if (newton) {
        // P R' P and P rho straight from the stage tile (P a mask there)
        D4 += sel(j < NU || j == VC, T);
      } else {
        // P R P and P R (c - u_ref) = P (R c + rho), independent of the chain
        // above (its instructions overlap it)
        D4 += PRP;
      }
      // A^T [W A | W d + q + s]: the part of S that needs no gains, issued
      // before the elimination
      const d4 SA = mmT<4>(At, D2, zero4());
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int r = 4 * q + g;
        if (j < NU) sr.G[r * GS + j] = D4[q] + ((r == j) ? 1.0 : 0.0) - Pt[q];
        if (j < NX) sr.G[r * GS + NU + j] = D5[q];
        if (j == VC) sr.G[r * GS + NU + NX] = D5[q] + D4[q];
      }
      wsync();
      // Gauss-Jordan elimination (H is SPD: no pivoting) of [H | Hwx | hw]
      // (and, for Newton steps, which keep H^-1, of [H | I] beside it): lane
      // 16 R + c holds column c of H (c < NU, the same in every row R) or
      // right-hand side 4 R + c - NU (Hwx columns 0..12, hw as 13 = VC;
      // identity columns 0..11); afterwards the right-hand sides are
      // H^-1 Hwx, H^-1 hw (and H^-1).
      static_assert(NU == 12, "row elimination is written for 12 inputs");
      const int hc = lane & 15, rhs = 4 * (lane >> 4) + hc - NU;
      const bool is_h = hc < NU;
      double col[NU];
#pragma unroll
      for (int r = 0; r < NU; ++r)
        col[r] = (is_h || rhs <= NX) ? sr.G[r * GS + (is_h ? hc : NU + rhs)] : 0.0;
      if constexpr (!newton && !ELEM) {
        gj_rows(col, unit);
      } else {
        double icol[NU];
#pragma unroll
        for (int r = 0; r < NU; ++r) icol[r] = is_h ? col[r] : ((r == rhs) ? 1.0 : 0.0);
        gj_rows2(col, icol, unit);
        if (!is_h && rhs < NU) {
#pragma unroll
          for (int r = 0; r < NU; ++r) sr.HI[r * 16 + rhs] = icol[r];
        }
      }
      if (!is_h && rhs <= NX) {
#pragma unroll
        for (int r = 0; r < NU; ++r) sr.KK[r * 16 + rhs] = -col[r];
      }
      wsync();
      d4 KK;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 4 * q + g;
        KK[q] = (r < NU && (j < NX || j == VC)) ? sr.KK[r * 16 + j] : 0.0;   // [K | kap]
      }
      if constexpr (!ELEM) {
        // K row-major (row r at NX r) for the rollout; rows 4q + g, q < 3, are
        // the 12 input rows (kap goes to its own vector)
        if (j < NX) {
#pragma unroll
          for (int q = 0; q < 3; ++q) prK[(size_t)k * TS_K + (4 * q + g) * NX + j] = KK[q];
        }
        vec_store(prkap + (size_t)k * NU, NU, KK);
        if (newton) {
          d4 HI;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = 4 * q + g;
            HI[q] = (r < NU && j < NU) ? sr.HI[r * 16 + j] : 0.0;
          }
          st_map(prL + (size_t)k * TS_L, TS_L, mL, HI);
          st_map(prH + (size_t)k * TS_H, TS_H, mH, D5);
        }
      } else {
        d4 HI;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = 4 * q + g;
          HI[q] = (r < NU && j < NU) ? sr.HI[r * 16 + j] : 0.0;
        }
        // the stage's closed-loop map [A + Bp K | d + Bp kap] with a 1 at
        // (13, 13), composed after the chunk's map; the reachability term
        // grows by A_E Bp H^-1 Bp^T A_E^T (A_E before the composition)
        const d4 BpT = mmT<3>(Pt, BT, zero4());    // (B P)^T = P B^T
        const d4 LK = mmT<3>(BpT, KK, zero4());    // [Bp K | Bp kap]
        d4 Ah;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = 4 * q + g;
          Ah[q] = (j < NX) ? At[q] + LK[q]
                           : ((j == VC) ? ((r < NX) ? LK[q] + D1[q] : (r == VC ? 1.0 : 0.0)) : 0.0);
        }
        const d4 ZT = mmT<4>(Bp, TE, zero4());     // (A_E Bp)^T
        const d4 Y = mmT<3>(HI, ZT, zero4());      // H^-1 (A_E Bp)^T
        CE = mmT<3>(ZT, Y, CE);
        TE = mmT<4>(Ah, TE, zero4());
      }
      // S = A^T W A + Hwx^T K, s = A^T (W d + q + s) + Hwx^T kap
      Sn = mmT<3>(sel(j < NX, D5), KK, SA);
      // keep S exactly symmetric: its rounding is not, and an asymmetric part
      // is carried back through the open-loop A and grows along the horizon
#pragma unroll
      for (int q = 0; q < 4; ++q) sr.ST[(4 * q + g) * 17 + j] = Sn[q];
      wsync();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 4 * q + g;
        if (r < NX && j < NX) Sn[q] = 0.5 * (Sn[q] + sr.ST[j * 17 + r]);
      }
      if (mode == Mode::EQ && !ELEM) st_map(prS + (size_t)k * TS_S, TS_S, mS, Sn);
      wsync();
    } else {
      // second right-hand side of the stored Newton matrix (d = 0, so
      // W d + q + s = q + s)
      const d4 wv = sel(j == VC, om + Ss);
      d4 hw = mmT<4>(Bp, wv, zero4());
      hw += sel(j == VC, T);
      const d4 kap = -mmT<3>(HIs, hw, zero4());
      vec_store(prkap + (size_t)k * NU, NU, kap);
      Sn = mmT<4>(At, wv, zero4());
      Sn = mmT<3>(HXs, kap, Sn);
    }
    Ss = Sn;
  }
  if constexpr (ELEM) {
    *TEo = TE;
    *CEo = CE;
  }
  return Ss;
}

// Forward rollout after the backward recursion (all N stages).
template <Mode mode, bool LONG>
__device__ __attribute__((always_inline)) inline void forward(const Ctx& C, Sh& sh) {
  const int N = __builtin_amdgcn_readfirstlane(C.N);
  const int lane = lane_id();
  constexpr bool newton = (mode == Mode::NEWTON);
  const gcf pA = uni(C.A), pB = uni(C.B), pe = uni(C.e);
  const GMEM uint8_t* pct = uni(C.contact);
  const gd prT = uni(C.rT), prK = uni(C.rK), prkap = uni(C.rkap), prx = uni(C.rx),
           pru = uni(C.ru), prdx = uni(C.rdx), prdu = uni(C.rdu);
  // forward rollout: w = K x + kap, u = P^T w + c (P from the stage tile;
  // the stance mask for Newton steps), x' = A x + B u + e.  It is a chain of
  // 13-vector products, so it runs on the vector units: lane i of every
  // 16-lane row holds x_i, w_i, u_i (the rows identical) with row i of K, A,
  // B and column i of P, and each product is a block of fused multiply-adds
  // whose vector factor arrives by DPP row broadcast.  The stage data is
  // fetched a stage ahead (unconditionally, so every path back to the loop
  // head has issued the same loads); u_k and x_{k+1} collect in LDS (the
  // costate buffers, free here) and are copied out after the loop.
  gd xout = newton ? prdx : prx;
  gd uout = newton ? prdu : pru;
  const StageBufs<LONG> sb(sh, C);
  const int fi = lane & 15;
  const int ix = clampi(fi, NX - 1), iu = clampi(fi, NU - 1);
  const gcf pev = pe ? pe : pA;   // a valid address when there is no e
  struct FwdRaw {
    double kr[NX];   // K[i][0..12]
    double p6[6];    // P[6 (i / 6) + a][i], a = 0..5 (equality passes)
    double c, kap;
    float a[NX], b[NU], e;
    int ct;
  };
  auto ffetch = [&](int k, FwdRaw& s) {
    const gcd kr = prK + (size_t)k * TS_K + iu * NX;
#pragma unroll
    for (int r = 0; r < NX; ++r) s.kr[r] = kr[r];
    s.kap = prkap[(size_t)k * NU + iu];
    if (!newton) {
      // column iu of P is nonzero only inside its contact's block
      const gcd tt = prT + (size_t)k * TS_T + (iu / 6) * 42;
#pragma unroll
      for (int a = 0; a < 6; ++a) s.p6[a] = tt[a * 6 + iu % 6];
      s.c = tt[36 + iu % 6];
    }
    const gcf ar = pA + (size_t)k * NX * NX + ix * NX;
#pragma unroll
    for (int r = 0; r < NX; ++r) s.a[r] = ar[r];
    const gcf br = pB + (size_t)k * NX * NU + ix * NU;
#pragma unroll
    for (int r = 0; r < NU; ++r) s.b[r] = br[r];
    s.e = pev[pe ? (size_t)k * NX + ix : 0];
    s.ct = newton ? (int)pct[k * 2 + iu / 6] : 0;
  };
  double xv = 0.0;   // x_k, entry fi
  if (!newton) xv = (double)uni(C.x0)[ix];
  FwdRaw fr;
  ffetch(0, fr);
  pin_memory();
  for (int k = 0; k < N; ++k) {
    double kr[NX], pc[NU], a[NX], b[NU];
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      kr[r] = fr.kr[r];
      a[r] = (double)fr.a[r];
    }
#pragma unroll
    for (int r = 0; r < NU; ++r) {
      pc[r] = (newton || r / 6 != iu / 6) ? 0.0 : fr.p6[r % 6];
      b[r] = (double)fr.b[r];
    }
    const double kap = fr.kap, cc = newton ? 0.0 : fr.c;
    const double ee = (!newton && pe) ? (double)fr.e : 0.0;
    const bool stance = fr.ct != 0;
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      pin(kr[r]);
      pin(a[r]);
    }
#pragma unroll
    for (int r = 0; r < NU; ++r) {
      pin(pc[r]);
      pin(b[r]);
    }
    pin_memory();
    ffetch(k + 1 < N ? k + 1 : k, fr);
    const double w = dot_row_bcast13(xv, kr, kap);
    const double u = newton ? (stance ? w : 0.0) : dot_row_bcast12(w, pc, cc);
    double xn = dot_row_bcast13(xv, a, ee);
    xn = dot_row_bcast12(u, b, xn);
    if (lane < NU) sb.GV[k * 16 + fi] = u;
    if (lane < NX) sb.PV[k * 16 + fi] = xn;
    xv = xn;
  }
  bufsync<LONG>();
  if (lane < NX) xout[lane] = newton ? 0.0 : (double)uni(C.x0)[lane];
  for (int e = lane; e < N * NU; e += W64) uout[e] = sb.GV[(e / NU) * 16 + e % NU];
  for (int e = lane; e < N * NX; e += W64) xout[NX + e] = sb.PV[(e / NX) * 16 + e % NX];
  gsync();
}

// The sequential recursion over the whole horizon (one wave), then the
// rollout.  Its stage loop is the one `backward` runs, written out here once
// more: compiled through the shared function, this hot loop took about 230
// more register moves per stage and its launch about 4 % longer.
template <Mode mode, bool factor, bool LONG>
__device__ __attribute__((noinline)) void riccati_t(const Ctx& C, Sh& sh, gcd rcvec, int ktop) {
  const int N = __builtin_amdgcn_readfirstlane(C.N);
  ktop = (mode == Mode::EQ) ? __builtin_amdgcn_readfirstlane(ktop < N ? ktop : N) : N;
  gsync();
  build_tiles(C, mode == Mode::NEWTON, rcvec, ktop);
  gsync();
  const int lane = lane_id(), g = tg(), j = tj();
  constexpr bool newton = (mode == Mode::NEWTON);
  const gcf pA = uni(C.A), pB = uni(C.B), pxr = uni(C.x_ref), pe = uni(C.e), pur = uni(C.u_ref);
  const GMEM uint8_t* pct = uni(C.contact);
  const GMEM int32_t* pfc = uni(C.faces);
  const gd prT = uni(C.rT), prK = uni(C.rK), prL = uni(C.rL), prH = uni(C.rHwx), prS = uni(C.rS);
  const gd prkap = uni(C.rkap), prx = uni(C.rx), pru = uni(C.ru), prdx = uni(C.rdx),
           prdu = uni(C.rdu);
  // the diagonal weights where this lane uses them
  const double Qj = C.Q[clampi(j, NX - 1)];
  d4 Qr, Rr;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    Qr[q] = C.Q[clampi(4 * q + g, NX - 1)];
    Rr[q] = C.R[clampi(4 * q + g, NU - 1)];
  }
  // maps of the stage blocks this variant moves
  const uint32_t mT = map_T();
  const uint32_t mS = map_S(true);
  const uint32_t mL = map_rect(NU, NU), mH = map_rect(NU, NX);
  auto fetch = [&](int k, BackRaw& s) {
    gather(pA + (size_t)k * NX * NX, false, NX, NX, s.a);
    gather(pB + (size_t)k * NX * NU, true, NX, NU, s.bt);
    gatherv(pxr + (size_t)k * NX, NX, s.xr);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      s.ev[q] = 0.f;
      s.ur[q] = 0.f;
      s.xn[q] = 0.0;
    }
    if (!newton && pe) gatherv(pe + (size_t)k * NX, NX, s.ev);
    if (!newton && pur) gatherv(pur + (size_t)k * NU, NU, s.ur);
    if (newton) {
#pragma unroll
      for (int q = 0; q < 4; ++q) s.xn[q] = prx[(size_t)(k + 1) * NX + clampi(4 * q + g, NX - 1)];
    }
    s.T = ld_map(prT + (size_t)k * TS_T, TS_T, mT);
    if (newton && !factor) {
      s.HI = ld_map(prL + (size_t)k * TS_L, TS_L, mL);
      s.HX = ld_map(prH + (size_t)k * TS_H, TS_H, mH);
    } else {
      s.HI = s.HX = zero4();
    }
    s.ct = newton ? (int)pct[k * 2 + (j < NU ? j / 6 : 0)] : 0;
    s.c0 = __builtin_amdgcn_readfirstlane((int)pct[k * 2]);
    s.c1 = __builtin_amdgcn_readfirstlane((int)pct[k * 2 + 1]);
    s.f0 = newton ? 0 : __builtin_amdgcn_readfirstlane(pfc[k * 2]);
    s.f1 = newton ? 0 : __builtin_amdgcn_readfirstlane(pfc[k * 2 + 1]);
  };

  // value function of x_{k+1}: S in columns 0..12, s in VC
  d4 Ss = (ktop < N) ? ld_map(prS + (size_t)ktop * TS_S, TS_S, map_S(false)) : zero4();
  BackRaw raw;
  fetch(ktop > 0 ? ktop - 1 : 0, raw);
  for (int k = ktop - 1; k >= 0; --k) {
    // this stage's data
    const d4 At = cook(raw.a, false, NX, NX);
    const d4 BT = cook(raw.bt, true, NX, NU);
    const d4 T = raw.T, HIs = raw.HI, HXs = raw.HX;
    d4 om, ev, ur;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = 4 * q + g;
      const bool vr = (j == VC && r < NX);
      const double xr = (double)raw.xr[q];
      om[q] = vr ? (newton ? Qr[q] * (raw.xn[q] - xr) : -Qr[q] * xr) : 0.0;
      ev[q] = vr ? (double)raw.ev[q] : 0.0;
      ur[q] = (j == VC && r < NU) ? (double)raw.ur[q] : 0.0;
    }
    const d4 Pt = newton ? mask_tile(raw.ct) : sel(j < NU, T);
    const uint32_t unit = null_inputs(raw.c0, raw.c1, raw.f0, raw.f1, newton);
    pin(At); pin(BT); pin(T); pin(om); pin(ev); pin(ur); pin(Pt);
    if (newton && !factor) { pin(HIs); pin(HXs); }
    pin_memory();
    if (k > 0) fetch(k - 1, raw);

    // [Bp | 0 | d] = B [P | 0 | c] + [0 | 0 | e]
    const d4 yc = (!newton && j == VC) ? T : Pt;
    d4 D1 = mmT<3>(BT, yc, ev);
    d4 PRP = zero4();
    if (!newton && factor) {
      d4 RP;
#pragma unroll
      for (int q = 0; q < 4; ++q) RP[q] = (j < NU && 4 * q + g < NU) ? Rr[q] * T[q] : 0.0;
      const d4 Py = (j < NU) ? T : sel(j == VC, T - ur);
      PRP = mmT<3>(RP, Py, zero4());
    }
    const d4 Bp = sel(j < NU, D1);
    d4 Sn;
    if (factor) {
      d4 Wt;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        Wt[q] = (j < NX) ? Ss[q] + ((4 * q + g == j) ? Qj : 0.0) : 0.0;
      const d4 yA = (j < NX) ? At : sel(j == VC, D1);
      d4 D2 = mmT<4>(Wt, yA, zero4());      // [W A | W d]
      if (j == VC) D2 += om + Ss;            // [W A | W d + q + s]
      const d4 D3 = mmT<4>(Wt, Bp, zero4()); // W Bp
      d4 D4 = mmT<4>(Bp, D3, zero4());       // Bp^T W Bp
      const d4 D5 = mmT<4>(Bp, D2, zero4()); // [Hwx | Bp^T (W d + q + s)]
      if (newton) {
        // P R' P and P rho straight from the stage tile (P a mask there)
        D4 += sel(j < NU || j == VC, T);
      } else {
        // P R P and P R (c - u_ref) = P (R c + rho), independent of the chain
        // above (its instructions overlap it)
        D4 += PRP;
      }
      // A^T [W A | W d + q + s]: the part of S that needs no gains, issued
      // before the elimination
      const d4 SA = mmT<4>(At, D2, zero4());
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int r = 4 * q + g;
        if (j < NU) sh.r.G[r * GS + j] = D4[q] + ((r == j) ? 1.0 : 0.0) - Pt[q];
        if (j < NX) sh.r.G[r * GS + NU + j] = D5[q];
        if (j == VC) sh.r.G[r * GS + NU + NX] = D5[q] + D4[q];
      }
      wsync();
      // Gauss-Jordan elimination (H is SPD: no pivoting) of [H | Hwx | hw]
      // (and, for Newton steps, which keep H^-1, of [H | I] beside it): lane
      // 16 R + c holds column c of H (c < NU, the same in every row R) or
      // right-hand side 4 R + c - NU (Hwx columns 0..12, hw as 13 = VC;
      // identity columns 0..11); afterwards the right-hand sides are
      // H^-1 Hwx, H^-1 hw (and H^-1).
      static_assert(NU == 12, "row elimination is written for 12 inputs");
      const int hc = lane & 15, rhs = 4 * (lane >> 4) + hc - NU;
      const bool is_h = hc < NU;
      double col[NU];
#pragma unroll
      for (int r = 0; r < NU; ++r)
        col[r] = (is_h || rhs <= NX) ? sh.r.G[r * GS + (is_h ? hc : NU + rhs)] : 0.0;
      if constexpr (!newton) {
        gj_rows(col, unit);
      } else {
        double icol[NU];
#pragma unroll
        for (int r = 0; r < NU; ++r) icol[r] = is_h ? col[r] : ((r == rhs) ? 1.0 : 0.0);
        gj_rows2(col, icol, unit);
        if (!is_h && rhs < NU) {
#pragma unroll
          for (int r = 0; r < NU; ++r) sh.r.HI[r * 16 + rhs] = icol[r];
        }
      }
      if (!is_h && rhs <= NX) {
#pragma unroll
        for (int r = 0; r < NU; ++r) sh.r.KK[r * 16 + rhs] = -col[r];
      }
      wsync();
      d4 KK;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 4 * q + g;
        KK[q] = (r < NU && (j < NX || j == VC)) ? sh.r.KK[r * 16 + j] : 0.0;   // [K | kap]
      }
      // K row-major (row r at NX r) for the rollout; rows 4q + g, q < 3, are
      // the 12 input rows (kap goes to its own vector)
      if (j < NX) {
#pragma unroll
        for (int q = 0; q < 3; ++q) prK[(size_t)k * TS_K + (4 * q + g) * NX + j] = KK[q];
      }
      vec_store(prkap + (size_t)k * NU, NU, KK);
      if (newton) {
        d4 HI;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = 4 * q + g;
          HI[q] = (r < NU && j < NU) ? sh.r.HI[r * 16 + j] : 0.0;
        }
        st_map(prL + (size_t)k * TS_L, TS_L, mL, HI);
        st_map(prH + (size_t)k * TS_H, TS_H, mH, D5);
      }
      // S = A^T W A + Hwx^T K, s = A^T (W d + q + s) + Hwx^T kap
      Sn = mmT<3>(sel(j < NX, D5), KK, SA);
      // keep S exactly symmetric: its rounding is not, and an asymmetric part
      // is carried back through the open-loop A and grows along the horizon
#pragma unroll
      for (int q = 0; q < 4; ++q) sh.r.ST[(4 * q + g) * 17 + j] = Sn[q];
      wsync();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 4 * q + g;
        if (r < NX && j < NX) Sn[q] = 0.5 * (Sn[q] + sh.r.ST[j * 17 + r]);
      }
      if (mode == Mode::EQ) st_map(prS + (size_t)k * TS_S, TS_S, mS, Sn);
      wsync();
    } else {
      // second right-hand side of the stored Newton matrix (d = 0, so
      // W d + q + s = q + s)
      const d4 wv = sel(j == VC, om + Ss);
      d4 hw = mmT<4>(Bp, wv, zero4());
      hw += sel(j == VC, T);
      const d4 kap = -mmT<3>(HIs, hw, zero4());
      vec_store(prkap + (size_t)k * NU, NU, kap);
      Sn = mmT<4>(At, wv, zero4());
      Sn = mmT<3>(HXs, kap, Sn);
    }
    Ss = Sn;
  }

  forward<mode, LONG>(C, sh);
}

// ---------------------------------------- associative scan over the horizon
//
// The backward recursion composes one map of the value function per stage,
// and that composition is associative.  With the horizon [0, ktop) cut into
// chunks, each chunk's composition (its summary) is formed on its own, the
// value functions at the chunk boundaries follow from the summaries alone,
// from the last chunk back to the first, and every chunk then runs the
// ordinary recursion from its boundary value, all chunks at once.  The
// summary of stages [k0, k1), from a zero value at x_{k1}, is
//   A_E, b_E  the closed-loop affine map from x_{k0} to x_{k1} (TE),
//   C_E       its reachability term, the sum of A' Bp H^-1 Bp^T A'^T (CE),
//   S_E, s_E  the value function of x_{k0} (SE),
// and the value function at x_{k0} for a value (S, s) at x_{k1} is, with
// J = S + Q and eta = -(s + q_{k1-1}) (the cost of x_{k1} included),
//   G = (J^-1 + C_E)^-1,   S_0 = A_E^T G A_E + S_E,
//   s_0 = s_E - A_E^T (I - G C_E)(eta - J b_E).
// The recursion is the paper's horizon-parallel treatment (Sec. III) applied
// to the LQ solve of the refinement: depth about 3 N / W + W stage steps for
// W chunks instead of N.  One wave per chunk: the problem's first wave runs
// the refinement; the others (helpers) take the scan's commands at the
// workgroup barrier and run the summaries and recursions of their chunks.

constexpr int SCAN_WMAX = 8;       // chunks (waves) per problem
constexpr int SCAN_MIN_CHUNK = 4;  // fewer stages per chunk: sequential
enum { SCAN_EXIT = 0, SCAN_EQ = 1, SCAN_NEWTON = 2 };
struct ScanCtl {
  int op, nch;
  int bounds[SCAN_WMAX + 1];
};
constexpr int TILE_D = 256;   // doubles of a register tile kept in LDS (lane-major)

__shared__ ScanCtl scan_ctl;
extern __shared__ __attribute__((aligned(16))) double scan_dyn[];

// Dynamic LDS of a scanning workgroup with W waves: the helpers' hand-off
// buffers, three summary tiles per chunk and a boundary value per chunk.
struct ScanLds {
  ShR* shr;
  double* exch;
  double* bnd;
};
__device__ inline ScanLds scan_lds(int W) {
  ScanLds L;
  L.shr = reinterpret_cast<ShR*>(scan_dyn);
  L.exch = scan_dyn + (size_t)(W - 1) * (sizeof(ShR) / 8);
  L.bnd = L.exch + (size_t)W * 3 * TILE_D;
  return L;
}

__device__ inline void st_tile_lds(double* base, const d4& t) {
  const int l = lane_id();
#pragma unroll
  for (int q = 0; q < 4; ++q) base[l * 4 + q] = t[q];
}
__device__ inline d4 ld_tile_lds(const double* base) {
  const int l = lane_id();
  d4 t;
#pragma unroll
  for (int q = 0; q < 4; ++q) t[q] = base[l * 4 + q];
  return t;
}

__device__ inline double readlane_d(double v, int l) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Inverse of the SPD 13 x 13 block of a tile by Gauss-Jordan elimination
// without pivoting: lane c < 13 holds column c of the matrix, lane 16 + c
// column c of the identity; each pivot's column reaches every lane by lane
// reads.  buf: 256 doubles of LDS.
__device__ d4 inv13(const d4& M, double* buf) {
  const int lane = lane_id(), g = tg(), j = tj();
#pragma unroll
  for (int q = 0; q < 4; ++q) buf[(4 * q + g) * 16 + j] = M[q];
  wsync();
  const int c = lane & 15;
  const bool mat = lane < NX, idn = lane >= 16 && lane < 16 + NX;
  double col[NX];
#pragma unroll
  for (int r = 0; r < NX; ++r) col[r] = mat ? buf[r * 16 + c] : ((idn && r == c) ? 1.0 : 0.0);
  wsync();
#pragma unroll
  for (int pv = 0; pv < NX; ++pv) {
    double m[NX];
#pragma unroll
    for (int r = 0; r < NX; ++r) m[r] = readlane_d(col[r], pv);
    const double rp = col[pv] * recip(m[pv]);
#pragma unroll
    for (int r = 0; r < NX; ++r)
      if (r != pv) col[r] = fma(-m[r], rp, col[r]);
    col[pv] = rp;
  }
  if (idn) {
#pragma unroll
    for (int r = 0; r < NX; ++r) buf[r * 16 + c] = col[r];
  }
  wsync();
  d4 R;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = 4 * q + g;
    R[q] = (r < NX && j < NX) ? buf[r * 16 + j] : 0.0;
  }
  wsync();
  return R;
}

// S exactly symmetric on its 13 x 13 block (the average with its transpose).
__device__ inline d4 symmetrize(d4 S, double* buf) {
  const int g = tg(), j = tj();
#pragma unroll
  for (int q = 0; q < 4; ++q) buf[(4 * q + g) * 17 + j] = S[q];
  wsync();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = 4 * q + g;
    if (r < NX && j < NX) S[q] = 0.5 * (S[q] + buf[j * 17 + r]);
  }
  wsync();
  return S;
}

// Value function [S_0 | s_0] at x_{k0} of a chunk with summary (TE, CE, SE)
// for the value V = [S | s] at x_{k1}; om holds q_{k1-1} in column VC.
__device__ d4 combine_value(const d4& TE, const d4& CE, const d4& SE, const d4& V, const d4& om,
                            double Qj, double* buf) {
  const int g = tg(), j = tj();
  d4 J, eta, E13;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = 4 * q + g;
    J[q] = (j < NX) ? V[q] + ((r == j) ? Qj : 0.0) : 0.0;
    eta[q] = (j == VC && r < NX) ? -(V[q] + om[q]) : 0.0;
    E13[q] = (r == VC && j == VC) ? 1.0 : 0.0;
  }
  const d4 Ji = inv13(J, buf);
  d4 X;
#pragma unroll
  for (int q = 0; q < 4; ++q) X[q] = (j < NX) ? Ji[q] + CE[q] : 0.0;
  const d4 G = inv13(X, buf);
  // b_E (row 13 of TE) as column VC, then t = eta - J b_E, u = (I - G C_E) t
  d4 bE = mmT<4>(TE, E13, zero4());
#pragma unroll
  for (int q = 0; q < 4; ++q) bE[q] = (4 * q + g < NX) ? bE[q] : 0.0;
  const d4 t = eta - mmT<4>(J, bE, zero4());
  const d4 u = t - mmT<4>(G, mmT<4>(CE, t, zero4()), zero4());
  // A_E: the transpose of TE's 13 x 13 block
#pragma unroll
  for (int q = 0; q < 4; ++q) buf[(4 * q + g) * 16 + j] = TE[q];
  wsync();
  d4 AE;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = 4 * q + g;
    AE[q] = (r < NX && j < NX) ? buf[j * 16 + r] : 0.0;
  }
  wsync();
  const d4 GA = mmT<4>(G, AE, zero4());
  d4 S0 = mmT<4>(AE, GA, SE);                     // [A^T G A + S_E | s_E]
  S0 -= sel(j == VC, mmT<4>(AE, u, zero4()));     // s_E - A^T u
  return symmetrize(S0, buf);
}

// The backward recursion as a scan over the horizon (the problem's first
// wave; the helpers run scan_helper).  Falls back to the sequential recursion
// when the horizon is too short to cut.
template <Mode mode, bool LONG>
__device__ __attribute__((noinline)) void riccati_scan(const Ctx& C, Sh& sh, gcd rcvec, int ktop) {
  const int N = __builtin_amdgcn_readfirstlane(C.N);
  ktop = (mode == Mode::EQ) ? __builtin_amdgcn_readfirstlane(ktop < N ? ktop : N) : N;
  gsync();
  build_tiles(C, mode == Mode::NEWTON, rcvec, ktop);
  gsync();
  constexpr bool newton = (mode == Mode::NEWTON);
  const int lane = lane_id(), g = tg(), j = tj();
  const int W = (int)(blockDim.x >> 6);
  const int nch = __builtin_amdgcn_readfirstlane(
      ktop / SCAN_MIN_CHUNK < W ? ktop / SCAN_MIN_CHUNK : W);
  const d4 Vk = (ktop < N) ? ld_map(uni(C.rS) + (size_t)ktop * TS_S, TS_S, map_S(false)) : zero4();
  if (nch < 2) {
    backward<mode, true, LONG, false>(C, sh.r, 0, ktop, Vk, nullptr, nullptr);
    forward<mode, LONG>(C, sh);
    return;
  }
  const ScanLds L = scan_lds(W);
  if (lane == 0) {
    scan_ctl.op = newton ? SCAN_NEWTON : SCAN_EQ;
    scan_ctl.nch = nch;
    for (int w = 0; w <= nch; ++w) scan_ctl.bounds[w] = (int)(((long)w * ktop) / nch);
  }
  __syncthreads();   // the command reaches the helpers
  __syncthreads();   // the helpers' chunk summaries are in LDS
  // boundary values, from the last chunk back to the first (the first chunk's
  // summary is not needed: its recursion starts from the boundary value)
  const gcf pxr = uni(C.x_ref);
  const gd prx = uni(C.rx);
  const double Qj = C.Q[clampi(j, NX - 1)];
  double* buf = L.exch;   // the first chunk's summary slot, free
  d4 V = Vk;
  st_tile_lds(L.bnd + (size_t)(nch - 1) * TILE_D, V);
  for (int w = nch - 1; w >= 1; --w) {
    const int k1 = __builtin_amdgcn_readfirstlane((int)(((long)(w + 1) * ktop) / nch));
    d4 om;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = 4 * q + g;
      const int rc = clampi(r, NX - 1);
      const double xr = (double)pxr[(size_t)(k1 - 1) * NX + rc];
      const double Qr = C.Q[rc];
      om[q] = (j == VC && r < NX) ? (newton ? Qr * (prx[(size_t)k1 * NX + rc] - xr) : -Qr * xr)
                                  : 0.0;
    }
    const double* ex = L.exch + (size_t)w * 3 * TILE_D;
    V = combine_value(ld_tile_lds(ex), ld_tile_lds(ex + TILE_D), ld_tile_lds(ex + 2 * TILE_D), V,
                      om, Qj, buf);
    st_tile_lds(L.bnd + (size_t)(w - 1) * TILE_D, V);
  }
  __syncthreads();   // the boundary values reach the helpers
  backward<mode, true, LONG, false>(C, sh.r, 0, (int)(ktop / nch), V, nullptr, nullptr);
  __syncthreads();   // every chunk's gains and values are stored
  forward<mode, LONG>(C, sh);
}

// A helper wave of a scanning workgroup: summary and recursion of its chunk
// for every scan command, until the first wave releases it.
template <bool LONG>
__device__ __attribute__((noinline)) void scan_helper(const Ctx& C) {
  const int wave = (int)(threadIdx.x >> 6), W = (int)(blockDim.x >> 6);
  const ScanLds L = scan_lds(W);
  ShR& sr = L.shr[wave - 1];
  for (;;) {
    __syncthreads();   // a command
    const int op = __builtin_amdgcn_readfirstlane(scan_ctl.op);
    if (op == SCAN_EXIT) return;
    const int nch = __builtin_amdgcn_readfirstlane(scan_ctl.nch);
    const bool mine = wave < nch;
    const int k0 = mine ? __builtin_amdgcn_readfirstlane(scan_ctl.bounds[wave]) : 0;
    const int k1 = mine ? __builtin_amdgcn_readfirstlane(scan_ctl.bounds[wave + 1]) : 0;
    if (mine) {
      d4 TE, CE, SE;
      if (op == SCAN_EQ)
        SE = backward<Mode::EQ, true, LONG, true>(C, sr, k0, k1, zero4(), &TE, &CE);
      else
        SE = backward<Mode::NEWTON, true, LONG, true>(C, sr, k0, k1, zero4(), &TE, &CE);
      double* ex = L.exch + (size_t)wave * 3 * TILE_D;
      st_tile_lds(ex, TE);
      st_tile_lds(ex + TILE_D, CE);
      st_tile_lds(ex + 2 * TILE_D, SE);
    }
    __syncthreads();   // summaries written
    __syncthreads();   // boundary values written
    if (mine) {
      const d4 V = ld_tile_lds(L.bnd + (size_t)wave * TILE_D);
      if (op == SCAN_EQ)
        backward<Mode::EQ, true, LONG, false>(C, sr, k0, k1, V, nullptr, nullptr);
      else
        backward<Mode::NEWTON, true, LONG, false>(C, sr, k0, k1, V, nullptr, nullptr);
    }
    __syncthreads();   // chunk recursions done
  }
}

// Releases the helpers of a scanning workgroup (the first wave, once).
__device__ inline void scan_release() {
  if (lane_id() == 0) scan_ctl.op = SCAN_EXIT;
  __syncthreads();
}
template <bool LONG>
__device__ void riccati(const Ctx& C, Sh& sh, Mode mode, bool factor, gcd rcvec, int ktop) {
  if (blockDim.x > W64 && factor) {   // a scanning workgroup
    if (mode == Mode::EQ) riccati_scan<Mode::EQ, LONG>(C, sh, rcvec, ktop);
    else riccati_scan<Mode::NEWTON, LONG>(C, sh, rcvec, ktop);
    return;
  }
  if (mode == Mode::EQ) riccati_t<Mode::EQ, true, LONG>(C, sh, rcvec, ktop);
  else if (factor) riccati_t<Mode::NEWTON, true, LONG>(C, sh, rcvec, ktop);
  else riccati_t<Mode::NEWTON, false, LONG>(C, sh, rcvec, ktop);
}

// Costates p_{k+1} = Q (x_{k+1} - r_k) + A_{k+1}^T p_{k+2} and the reduced
// gradient g_k = R (u_k - u_ref_k) + B_k^T p_{k+1}.  The terms that need no
// costate are formed first, in parallel, into LDS.  The recursion is a chain
// of 13-vector products, so it runs on the vector units rather than the
// matrix cores (where a 16 x 16 tile product per stage would carry one useful
// column): lane i of every 16-lane row holds entry i of p (the rows
// identical) and column i of A_{k+1} and B_k, and each product is 13 fused
// multiply-adds whose other factor, p_r, arrives by row broadcast.  Columns
// are fetched two stages ahead (unconditionally, stage index clamped, loop
// left as a whole, no global store inside: each stage waits for its own
// loads only); p and g stay in LDS until the chain is done.  Returns the
// state-side magnitude max |Q (x_{k+1} - r_k)|, |p|, |p - Q (x_{k+1} - r_k)|
// (= |A^T p_{k+2}|) over all stages, which the KKT scaling needs.
template <bool LONG>
__device__ __attribute__((noinline)) double costates_grad(const Ctx& C, Sh& sh) {
  gsync();
  const StageBufs<LONG> sb(sh, C);
  const int lane = lane_id();
  const int N = __builtin_amdgcn_readfirstlane(C.N);
  const gcf pA = uni(C.A), pB = uni(C.B), pxr = uni(C.x_ref), pur = uni(C.u_ref);
  const gd prx = uni(C.rx), pru = uni(C.ru), prlam = uni(C.rlam), prg = uni(C.rg);
  for (int e = lane; e < N * NX; e += W64) {
    const int k = e / NX, i = e % NX;
    sb.PV[k * 16 + i] = C.Q[i] * (prx[(size_t)(k + 1) * NX + i] - (double)pxr[(size_t)k * NX + i]);
  }
  for (int e = lane; e < N * NU; e += W64) {
    const int k = e / NU, i = e % NU;
    const double ur = pur ? (double)pur[(size_t)k * NU + i] : 0.0;
    sb.GV[k * 16 + i] = C.R[i] * (pru[(size_t)k * NU + i] - ur);
  }
  bufsync<LONG>();
  const int i = lane & 15;
  const int ia = clampi(i, NX - 1), ib = clampi(i, NU - 1);
  struct ColRaw {
    float a[NX], b[NX];   // A_{k+1}[r][i], B_k[r][i]
  };
  // stage k needs A_{k+1} (for p_{k+1}) and B_k (for g_k); at k = N - 1 the
  // clamped A_N multiplies p_{N+1} = 0
  auto cfetch = [&](int k, ColRaw& s) {
    const gcf Ak = pA + (size_t)clampi(k + 1, N - 1) * NX * NX;
    const gcf Bk = pB + (size_t)k * NX * NU;
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      s.a[r] = Ak[r * NX + ia];
      s.b[r] = Bk[r * NU + ib];
    }
  };
  constexpr int CD = 2;
  ColRaw ring[CD];
#pragma unroll
  for (int d = 0; d < CD; ++d) {
    cfetch(N - 1 - d >= 0 ? N - 1 - d : 0, ring[d]);
    pin_memory();   // issued in ring order, as the loop issues them
  }
  double p = 0.0;   // p_{k+2}, entry i
  double tstate = 0.0;
  for (int k = N - 1;;) {
#pragma unroll
    for (int d = 0; d < CD; ++d, --k) {
      if (k < 0) goto chain_done;
      double a[NX], b[NX];
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        a[r] = (double)ring[d].a[r];
        b[r] = (double)ring[d].b[r];
      }
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        pin(a[r]);
        pin(b[r]);
      }
      pin_memory();
      cfetch(k - CD >= 0 ? k - CD : 0, ring[d]);
      const double qx = (i < NX) ? sb.PV[k * 16 + i] : 0.0;
      const double rg = (i < NU) ? sb.GV[k * 16 + i] : 0.0;
      p = dot_row_bcast13(p, a, qx);          // p_{k+1}
      const double gk = dot_row_bcast13(p, b, rg);
      if (i < NX) tstate = fmax(tstate, fmax(fabs(qx), fmax(fabs(p), fabs(p - qx))));
      if (lane < NX) sb.PV[k * 16 + i] = p;
      if (lane < NU) sb.GV[k * 16 + i] = gk;
    }
  }
chain_done:
  bufsync<LONG>();
  for (int e = lane; e < N * NX; e += W64) prlam[e] = sb.PV[(e / NX) * 16 + e % NX];
  for (int e = lane; e < N * NU; e += W64) prg[e] = sb.GV[(e / NU) * 16 + e % NU];
  gsync();
  return wave_max(tstate);
}

// Row data of one stance contact-stage (k, i) in registers: a lane owns a
// contact-stage and its 11 rows, so each row pass over the horizon issues its
// loads together and stores once (no store-then-load chains between rows).
__device__ inline void load_u6(gcd v, int k, int i, double x[6]) {
#pragma unroll
  for (int a = 0; a < 6; ++a) x[a] = v[k * NU + 6 * i + a];
}
__device__ inline void load_r(gcd v, size_t rb, double x[NROW]) {
#pragma unroll
  for (int r = 0; r < NROW; ++r) x[r] = v[rb + r];
}
__device__ inline void store_r(gd v, size_t rb, const double x[NROW]) {
#pragma unroll
  for (int r = 0; r < NROW; ++r) v[rb + r] = x[r];
}
// g_r u, h_r and the row scale of the contact's 11 rows
__device__ inline void rows_of(const Ctx& C, const double u[6], double gu[NROW], double hh[NROW],
                               double sc[NROW]) {
#pragma unroll
  for (int r = 0; r < NROW; ++r) {
    double g[6];
    wrench_row(r, C.mu, C.fz, C.tm, g, &hh[r]);
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < 6; ++a) acc += g[a] * u[a];
    gu[r] = acc;
    sc[r] = (r < 5) ? C.mg : C.tm;
  }
}

// Row multipliers of each stance contact from its face and the gradient, and
// the normalised KKT residuals of the current (u, x, p, mu).  Returns KKT.
__device__ __attribute__((noinline)) double multipliers_kkt(const Ctx& C, double res[PINMPC_NRES],
                                                           double term_state) {
  gsync();
  const int lane = lane_id();
  double r_ineq = 0.0, stat = 0.0, term = term_state, comp = 0.0, mumax = 0.0, neg = 0.0;
  for (int e = lane; e < C.N * 2; e += W64) {
    const int k = e >> 1, i = e & 1;
    const int st = k;
    // the contact-stage's inputs, gradient and multipliers in registers
    double u[6], g[6], mu[NROW];
    load_u6(C.ru, st, i, u);
    load_u6(C.rg, st, i, g);
#pragma unroll
    for (int r = 0; r < NROW; ++r) mu[r] = 0.0;
    gd mu_out = C.rmu + (st * 2 + i) * NROW;
    if (!C.contact[st * 2 + i]) {
      for (int a = 0; a < 6; ++a) r_ineq = fmax(r_ineq, fabs(u[a]) / C.mg);
      store_r(mu_out, 0, mu);
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
      // the four side rows are [+-1, 0, -mu] and [0, +-1, -mu]: with b = -g_f
      // and S = -b_z / mu the three-row systems are
      //   mu0 - mu1 = b_x,  mu2 - mu3 = b_y,  mu0 + mu1 + mu2 + mu3 = S
      // with the dropped multiplier zero, solved in closed form
      const double bx = -g[0], by = -g[1], S = g[2] / C.mu;
      double cand[4][4];
      cand[0][0] = 0.0;                    cand[0][1] = -bx;
      cand[0][2] = 0.5 * (S + bx + by);    cand[0][3] = 0.5 * (S + bx - by);
      cand[1][0] = bx;                     cand[1][1] = 0.0;
      cand[1][2] = 0.5 * (S - bx + by);    cand[1][3] = 0.5 * (S - bx - by);
      cand[2][0] = 0.5 * (S + by + bx);    cand[2][1] = 0.5 * (S + by - bx);
      cand[2][2] = 0.0;                    cand[2][3] = -by;
      cand[3][0] = 0.5 * (S - by + bx);    cand[3][1] = 0.5 * (S - by - bx);
      cand[3][2] = by;                     cand[3][3] = 0.0;
      double best = -1e300;
      int pick = 0;
#pragma unroll
      for (int drop = 0; drop < 4; ++drop) {
        double mn = 1e300;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (i != drop) mn = fmin(mn, cand[drop][i]);
        if (mn > best) {
          best = mn;
          pick = drop;
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        double v = cand[0][i];
#pragma unroll
        for (int d = 1; d < 4; ++d) v = (pick == d) ? cand[d][i] : v;
        mu[i] = v;
      }
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
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (code >> (8 + a) & 1) mu[5 + a] = -g[3 + a];
      else if (code >> (11 + a) & 1) mu[8 + a] = g[3 + a];
    }
    store_r(mu_out, 0, mu);
    // residual pieces
    double gm[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int r = 0; r < NROW; ++r) {
      double gg[6], hh;
      wrench_row(r, C.mu, C.fz, C.tm, gg, &hh);
      double gu = 0.0;
#pragma unroll
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
  // the state-side term norms (|Q (x - r)|, |p|, |A^T p|) come in as
  // term_state from the costate recursion, which holds them
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
__device__ __attribute__((noinline)) double dyn_residual(const Ctx& C) {
  gsync();
  const int lane = lane_id();
  double r = 0.0;
  for (int e = lane; e < C.N * NX; e += W64) {
    const int k = e / NX, i = e % NX;
    const int st = k;
    gcd x = C.rx + k * NX;
    gcf A = C.A + st * NX * NX + i * NX;
    gcf B = C.B + st * NX * NU + i * NU;
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
// hash of the new face set and, in *ktop, one past the last stage whose face
// changed (0: none did).
__device__ __attribute__((noinline)) uint64_t pdas_update(const Ctx& C, int* ktop) {
  gsync();
  const int lane = lane_id();
  uint64_t hsh = 0;
  int kch = 0;
  for (int e = lane; e < C.N * 2; e += W64) {
    const int k = e >> 1, i = e & 1;
    const int st = k;
    int code = 0;
    if (C.contact[st * 2 + i]) {
      gcd u = C.ru + st * NU + 6 * i;
      gcd mu = C.rmu + (st * 2 + i) * NROW;
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
    if (C.faces[st * 2 + i] != code) kch = k + 1;
    C.faces[st * 2 + i] = code;
    uint64_t v = (uint64_t)(code + 1) * 0x9E3779B97F4A7C15ull ^ ((uint64_t)(e + 1) * 0xC2B2AE3D27D4EB4Full);
    v ^= v >> 29;
    v *= 0xBF58476D1CE4E5B9ull;
    hsh ^= v;
  }
  wsync();
  *ktop = (int)wave_max((double)kch);
  return wave_xor(hsh);
}

// Faces from slack: rows whose slack is below tol * row scale.
__device__ __attribute__((noinline)) void faces_from_u(const Ctx& C, gcd u_src, double tol) {
  gsync();
  const int lane = lane_id();
  for (int e = lane; e < C.N * 2; e += W64) {
    const int k = e >> 1, i = e & 1;
    const int st = k;
    int code = 0;
    if (C.contact[st * 2 + i]) {
      gcd u = u_src + st * NU + 6 * i;
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
// costates, multipliers and residuals.  `ktop` < N: the faces of stages
// ktop..N-1 are those of the previous equality-constrained solve, whose tiles
// and factors are still in the scratch block.
// The pass's x is the FP64 rollout of its u, so its dynamics residual is
// rounding only: it is checked once, on the final trajectory, by the caller.
template <bool LONG>
__device__ __attribute__((noinline)) double eq_pass(const Ctx& C, Sh& sh, double res[PINMPC_NRES],
                                                   int ktop) {
  riccati<LONG>(C, sh, Mode::EQ, true, nullptr, ktop);
  const double ts = costates_grad<LONG>(C, sh);
  return multipliers_kkt(C, res, ts);
}

// Faces from the interior-point iterate (row active where z > s); returns an
// order-independent hash of the face set.
__device__ __attribute__((noinline)) uint64_t faces_from_zs(const Ctx& C) {
  gsync();
  const int lane = lane_id();
  uint64_t hsh = 0;
  for (int e = lane; e < C.N * 2; e += W64) {
    const int k = e >> 1, i = e & 1;
    int code = 0;
    if (C.contact[k * 2 + i]) {
      const size_t rb = (size_t)(k * 2 + i) * NROW;
      for (int r = 0; r < NROW; ++r)
        if (C.rz[rb + r] > C.rs[rb + r]) code |= (r < 5) ? (1 << r) : (1 << (8 + (r - 5)));
      if (face_apex(code)) code = (code & ~31) | FACE_APEX;
      for (int a = 0; a < 3; ++a)
        if ((code >> (8 + a) & 1) && (code >> (11 + a) & 1)) code &= ~(1 << (11 + a));
    }
    C.faces[k * 2 + i] = code;
    uint64_t v = (uint64_t)(code + 1) * 0x9E3779B97F4A7C15ull ^ ((uint64_t)(e + 1) * 0xC2B2AE3D27D4EB4Full);
    v ^= v >> 29;
    v *= 0xBF58476D1CE4E5B9ull;
    hsh ^= v;
  }
  wsync();
  return wave_xor(hsh);
}

// Work done by the refinement of one problem: equality-constrained passes
// (active-set, crossover and polish passes), interior-point iterations, and
// the stages whose backward recursion an equality pass factored (a pass that
// restarts at stage ktop factors ktop stages).
struct Counts {
  int eq, ipm, stf;
};

// Interior-point fallback.  Rows scaled by mg (force rows) and tau_max
// (moment rows).  Crossover: once the face guess z > s is the same after two
// consecutive iterations, one equality-constrained pass on those faces is
// tried (the iterate is kept aside and restored if it does not certify).
// Returns the number of iterations; *certified tells whether a crossover pass
// certified (then ru, rx, res and *kkt are that pass's), else the faces from
// z > s are left for the polish passes.
template <bool LONG>
__device__ __attribute__((noinline)) int ipm(const Ctx& C, Sh& sh, int maxit, double tol, Counts* cnt,
                   double res[PINMPC_NRES], double* kkt_out, bool* certified) {
  *certified = false;
  gsync();
  const int lane = lane_id();
  const int N = C.N;
  // number of stance rows
  int mloc = 0;
  for (int e = lane; e < N * 2; e += W64)
    if (C.contact[(e >> 1) * 2 + (e & 1)]) mloc += NROW;
  const double m = wave_sum((double)mloc);
  if (m == 0.0) return 0;
  gd rc = C.rdz;   // complementarity target
  // initial point: the current ru (the ADMM point) and its rollout in rx,
  // slacks at least 1, multipliers 1 (a start from the last active-set pass,
  // its slacks and multipliers floored at 1e-1 .. 1e-3, took as long or
  // longer: the early steps near the boundary are short); and the residuals
  // of that point
  double smz = 0.0, rpn = 0.0;
  for (int e = lane; e < N * 2; e += W64) {
    const int k = e >> 1, i = e & 1;
    if (!C.contact[k * 2 + i]) continue;
    const size_t rb = (size_t)e * NROW;
    double u[6], gu[NROW], hh[NROW], sc[NROW], sv[NROW], zv[NROW], cv[NROW];
    load_u6(C.ru, k, i, u);
    rows_of(C, u, gu, hh, sc);
#pragma unroll
    for (int r = 0; r < NROW; ++r) {
      sv[r] = fmax((hh[r] - gu[r]) / sc[r], 1.0);
      zv[r] = 1.0;
      rpn = fmax(rpn, fabs((gu[r] - hh[r]) / sc[r] + sv[r]));
      smz += sv[r] * zv[r];
      cv[r] = sv[r] * zv[r];
    }
    store_r(C.rs, rb, sv);
    store_r(C.rz, rb, zv);
    store_r(rc, rb, cv);
  }
  int it = 0;
  uint64_t hprev = 0;
  for (; it < maxit; ++it) {
    const double muv = wave_sum(smz) / m;
    rpn = wave_max(rpn);
    if (muv <= 1e-10 && rpn <= 1e-9) break;
    // predictor (affine target rc = s z)
    riccati<LONG>(C, sh, Mode::NEWTON, true, rc, C.N);
    double amax_s = 1.0, amax_z = 1.0;
    for (int e = lane; e < N * 2; e += W64) {
      const int k = e >> 1, i = e & 1;
      if (!C.contact[k * 2 + i]) continue;
      const size_t rb = (size_t)e * NROW;
      double u[6], du[6], gu[NROW], gdu[NROW], hh[NROW], sc[NROW], sv[NROW], zv[NROW];
      load_u6(C.ru, k, i, u);
      load_u6(C.rdu, k, i, du);
      load_r(C.rs, rb, sv);
      load_r(C.rz, rb, zv);
      rows_of(C, u, gu, hh, sc);
      rows_of(C, du, gdu, hh, sc);
      double dsv[NROW], dzv[NROW];
#pragma unroll
      for (int r = 0; r < NROW; ++r) {
        const double rp = (gu[r] - hh[r]) / sc[r] + sv[r];
        dsv[r] = -rp - gdu[r] / sc[r];
        dzv[r] = (-sv[r] * zv[r] - zv[r] * dsv[r]) / sv[r];
        if (dsv[r] < 0) amax_s = fmin(amax_s, -sv[r] / dsv[r]);
        if (dzv[r] < 0) amax_z = fmin(amax_z, -zv[r] / dzv[r]);
      }
      store_r(C.rds, rb, dsv);
      store_r(C.rmu, rb, dzv);    // affine dz kept in rmu scratch
    }
    const double aa = fmin(wave_min(amax_s), wave_min(amax_z));
    double sm = 0.0;
    for (int e = lane; e < N * 2; e += W64) {
      const int k = e >> 1, i = e & 1;
      if (!C.contact[k * 2 + i]) continue;
      const size_t rb = (size_t)e * NROW;
      double sv[NROW], zv[NROW], dsv[NROW], dzv[NROW];
      load_r(C.rs, rb, sv);
      load_r(C.rz, rb, zv);
      load_r(C.rds, rb, dsv);
      load_r(C.rmu, rb, dzv);
#pragma unroll
      for (int r = 0; r < NROW; ++r) sm += (sv[r] + aa * dsv[r]) * (zv[r] + aa * dzv[r]);
    }
    const double mu_aff = wave_sum(sm) / m;
    const double sigma = pow(mu_aff / muv, 3.0);
    // corrector target: s z + ds_aff dz_aff - sigma mu
    for (int e = lane; e < N * 2; e += W64) {
      const int k = e >> 1, i = e & 1;
      if (!C.contact[k * 2 + i]) continue;
      const size_t rb = (size_t)e * NROW;
      double sv[NROW], zv[NROW], dsv[NROW], dzv[NROW], cv[NROW];
      load_r(C.rs, rb, sv);
      load_r(C.rz, rb, zv);
      load_r(C.rds, rb, dsv);
      load_r(C.rmu, rb, dzv);
#pragma unroll
      for (int r = 0; r < NROW; ++r) cv[r] = sv[r] * zv[r] + dsv[r] * dzv[r] - sigma * muv;
      store_r(rc, rb, cv);
    }
    // corrector: same matrix, new right-hand side
    riccati<LONG>(C, sh, Mode::NEWTON, false, rc, C.N);
    amax_s = 1.0;
    amax_z = 1.0;
    for (int e = lane; e < N * 2; e += W64) {
      const int k = e >> 1, i = e & 1;
      if (!C.contact[k * 2 + i]) continue;
      const size_t rb = (size_t)e * NROW;
      double u[6], du[6], gu[NROW], gdu[NROW], hh[NROW], sc[NROW], sv[NROW], zv[NROW], cv[NROW];
      load_u6(C.ru, k, i, u);
      load_u6(C.rdu, k, i, du);
      load_r(C.rs, rb, sv);
      load_r(C.rz, rb, zv);
      load_r(rc, rb, cv);
      rows_of(C, u, gu, hh, sc);
      rows_of(C, du, gdu, hh, sc);
      double dsv[NROW], dzv[NROW];
#pragma unroll
      for (int r = 0; r < NROW; ++r) {
        const double rp = (gu[r] - hh[r]) / sc[r] + sv[r];
        dsv[r] = -rp - gdu[r] / sc[r];
        dzv[r] = (-cv[r] - zv[r] * dsv[r]) / sv[r];
        if (dsv[r] < 0) amax_s = fmin(amax_s, -sv[r] / dsv[r]);
        if (dzv[r] < 0) amax_z = fmin(amax_z, -zv[r] / dzv[r]);
      }
      store_r(C.rds, rb, dsv);
      store_r(C.rmu, rb, dzv);
    }
    const double a = fmin(1.0, 0.99 * fmin(wave_min(amax_s), wave_min(amax_z)));
    // step, and the residuals and affine target of the new point; a lane
    // updates the inputs of its own contact-stage (swing inputs stay 0)
    smz = 0.0;
    rpn = 0.0;
    for (int e = lane; e < N * 2; e += W64) {
      const int k = e >> 1, i = e & 1;
      if (!C.contact[k * 2 + i]) continue;
      const size_t rb = (size_t)e * NROW;
      double u[6], du[6], gu[NROW], hh[NROW], sc[NROW], sv[NROW], zv[NROW], dsv[NROW], dzv[NROW],
          cv[NROW];
      load_u6(C.ru, k, i, u);
      load_u6(C.rdu, k, i, du);
      load_r(C.rs, rb, sv);
      load_r(C.rz, rb, zv);
      load_r(C.rds, rb, dsv);
      load_r(C.rmu, rb, dzv);
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        u[t] += a * du[t];
        C.ru[k * NU + 6 * i + t] = u[t];
      }
      rows_of(C, u, gu, hh, sc);
#pragma unroll
      for (int r = 0; r < NROW; ++r) {
        sv[r] += a * dsv[r];
        zv[r] += a * dzv[r];
        rpn = fmax(rpn, fabs((gu[r] - hh[r]) / sc[r] + sv[r]));
        smz += sv[r] * zv[r];
        cv[r] = sv[r] * zv[r];
      }
      store_r(C.rs, rb, sv);
      store_r(C.rz, rb, zv);
      store_r(rc, rb, cv);
    }
    // states: loads of a group first, then its stores
    for (int e0 = lane; e0 < (N + 1) * NX; e0 += 4 * W64) {
      double xv[4], dv[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int e = e0 + t * W64;
        xv[t] = (e < (N + 1) * NX) ? C.rx[e] : 0.0;
        dv[t] = (e < (N + 1) * NX) ? C.rdx[e] : 0.0;
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int e = e0 + t * W64;
        if (e < (N + 1) * NX) C.rx[e] = xv[t] + a * dv[t];
      }
    }
    wsync();
    const uint64_t h = faces_from_zs(C);
    if (it >= 1 && h == hprev) {
      // the step buffers are free between iterations: keep the iterate there
      gsync();
      for (int e = lane; e < N * NU; e += W64) C.rdu[e] = C.ru[e];
      for (int e = lane; e < (N + 1) * NX; e += W64) C.rdx[e] = C.rx[e];
      const double kkt = eq_pass<LONG>(C, sh, res, N);
      ++cnt->eq;
      cnt->stf += N;
      if (kkt <= tol) {
        *kkt_out = kkt;
        *certified = true;
        return it + 1;
      }
      gsync();
      for (int e = lane; e < N * NU; e += W64) C.ru[e] = C.rdu[e];
      for (int e = lane; e < (N + 1) * NX; e += W64) C.rx[e] = C.rdx[e];
      wsync();
    }
    hprev = h;
  }
  faces_from_zs(C);
  return it;
}

// Active-set loop; returns true if certified.  cnt accumulates.
template <bool LONG>
__device__ bool active_set_loop(const Ctx& C, Sh& sh, int maxp, double tol, Counts* cnt,
                                double res[PINMPC_NRES], double* kkt_out,
                                bool* cycled = nullptr) {
  if (cycled) *cycled = false;
  uint64_t hist[8];
  for (int i = 0; i < 8; ++i) hist[i] = 0;
  int nh = 0;
  int ktop = C.N;   // the first pass solves the whole horizon
  for (int it = 0; it < maxp; ++it) {
    const double kkt = eq_pass<LONG>(C, sh, res, ktop);
    ++cnt->eq;
    cnt->stf += ktop < C.N ? ktop : C.N;
    *kkt_out = kkt;
    if (kkt <= tol) return true;
    const uint64_t h = pdas_update(C, &ktop);
    bool seen = false;
    for (int i = 0; i < 8; ++i) seen |= (hist[i] == h) && (i < nh || nh >= 8);
    if (seen) {
      if (cycled) *cycled = true;
      return false;
    }
    hist[nh & 7] = h;
    ++nh;
  }
  return false;
}

__device__ __attribute__((noinline)) void rollout_ru(const Ctx& C, Sh& sh) {
  gsync();
  // x = rollout of ru from x0, in FP64, into rx
  const int lane = lane_id();
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
__device__ __attribute__((noinline)) void admm_point(const Ctx& C, gcf zsrc, gcf sf, float tsc) {
  gsync();
  const int lane = lane_id();
  for (int e = lane; e < C.N * NU; e += W64) {
    const int k = e / NU, j = e % NU;
    const double sc = (j % 6 < 3) ? (double)sf[k] : (double)tsc;
    double v = (double)zsrc[((size_t)k * NSTATE) * NL + NX + j] * sc;
    if (!C.contact[k * 2 + j / 6]) v = 0.0;
    C.ru[k * NU + j] = v;
  }
  wsync();
}

// PHASE 1 runs every problem's active-set passes; a problem they do not
// certify (with the interior point enabled) is appended to ws.rlist and left
// to PHASE 2, which runs the interior point and the polish passes for the
// listed problems only (surplus blocks exit).  The slow problems thus start
// together instead of behind a second round of easy ones.
// The first wave releases a scanning workgroup's helpers on every way out.
template <bool SCAN>
struct ScanRelease {
  __device__ ~ScanRelease() {
    if constexpr (SCAN) scan_release();
  }
};

template <int PHASE, bool LONG, bool SCAN>
__global__ void __launch_bounds__(SCAN ? 64 * SCAN_WMAX : 64, 2) refine_kernel(Problem p, Workspace ws, float* out_u,
                                                    float* out_x, float* out_res,
                                                    int32_t* out_iters, int32_t* out_status,
                                                    int32_t* out_detail,
                                                    int admm_iters, int accel, int refine,
                                                    int pass_a, int ipm_max, int pass_c,
                                                    double tol, int pass_1) {
  __shared__ Sh sh;
  // the problem context lives in LDS: its pointers are loaded where they are
  // used instead of being held in registers across the whole kernel
  __shared__ Ctx C;
  int pb = blockIdx.x;
  if (PHASE == 2) {
    if ((int)blockIdx.x >= ws.rcount[0]) return;
    pb = ws.rlist[blockIdx.x];
  }
  if constexpr (SCAN) {
    // with the horizon scan the workgroup holds one wave per chunk: all but
    // the first take the scan's commands until the first releases them
    if (threadIdx.x >= W64) {
      scan_helper<LONG>(C);
      return;
    }
  }
  const ScanRelease<SCAN> release;
  const int lane = lane_id();
  if (lane == 0) {
  C.b = pb;
  C.n = p.n_max;
  C.N = horizon(p, C.b);
  const size_t s0 = (size_t)C.b * C.n;
  C.mu = p.mu[C.b];
  C.fz = p.fz_max[C.b];
  C.tm = p.tau_max[C.b];
  C.mg = weight_of(p, C.b);
  C.Q = (const LMEM double*)sh.Qd;
  C.R = (const LMEM double*)sh.Rd;
  C.A = (gcf)(p.A + s0 * NX * NX);
  C.B = (gcf)(p.B + s0 * NX * NU);
  C.e = p.e ? (gcf)(p.e + s0 * NX) : nullptr;
  C.x_ref = (gcf)(p.x_ref + s0 * NX);
  C.u_ref = p.u_ref ? (gcf)(p.u_ref + s0 * NU) : nullptr;
  C.x0 = (gcf)(p.x0 + (size_t)C.b * NX);
  C.contact = (const GMEM uint8_t*)(p.contact + s0 * 2);
  {
    const int n = C.n;
    gd blk = (gd)(ws.rblk + (size_t)C.b * refine_block_doubles(n));
    C.rT = blk;                       blk += (size_t)n * TS_T;
    C.rK = blk;                       blk += (size_t)n * TS_K;
    C.rL = blk;                       blk += (size_t)n * TS_L;
    C.rHwx = blk;                     blk += (size_t)n * TS_H;
    C.rS = blk;                       blk += (size_t)n * TS_S;
    C.rkap = blk;                     blk += (size_t)n * NU;
    C.ru = blk;                       blk += (size_t)n * NU;
    C.rlam = blk;                     blk += (size_t)n * NX;
    C.rg = blk;                       blk += (size_t)n * NU;
    C.rmu = blk;                      blk += (size_t)n * 2 * NROW;
    C.rs = blk;                       blk += (size_t)n * 2 * NROW;
    C.rz = blk;                       blk += (size_t)n * 2 * NROW;
    C.rds = blk;                      blk += (size_t)n * 2 * NROW;
    C.rdz = blk;                      blk += (size_t)n * 2 * NROW;
    C.rdu = blk;                      blk += (size_t)n * NU;
    C.rx = blk;                       blk += (size_t)(n + 1) * NX;
    C.rdx = blk;                      blk += (size_t)(n + 1) * NX;
    C.rPV = blk;                      blk += (size_t)n * 16;
    C.rGV = blk;   // inside the block only for n > PINMPC_NMAX (LONG)
    C.faces = (GMEM int32_t*)(ws.faces + s0 * 2);
  }
  }
  if (lane < NX) sh.Qd[lane] = p.Q[(size_t)pb * NX + lane];
  if (lane < NU) sh.Rd[lane] = p.R[(size_t)pb * NU + lane];
  wsync();
  const size_t s0 = (size_t)pb * p.n_max;
  const int N = C.N;

  // input checks: finiteness of the scalars and weights, then the bounds
  // (a friction coefficient must be positive: mu = 0 leaves the pyramid
  // without f_z >= 0 and its apex multipliers undefined), then finiteness of
  // this problem's stage data
  const int Nraw = horizon_raw(p, C.b);
  int nonfinite = !isfinite(C.mu) || !isfinite(C.fz) || !isfinite(C.tm) || !isfinite(C.mg);
  for (int j = 0; j < NX; ++j) nonfinite |= !isfinite(C.Q[j]);
  for (int j = 0; j < NU; ++j) nonfinite |= !isfinite(C.R[j]);
  int bad = 0;
  if (!nonfinite) {
    bad = !(C.mu > 0.0) || !(C.fz >= 0.0) || !(C.tm >= 0.0) || !(C.mg > 0.0) || Nraw < 1 ||
          Nraw > C.n;
    for (int j = 0; j < NX; ++j) bad |= !(C.Q[j] > 0.0);
    for (int j = 0; j < NU; ++j) bad |= !(C.R[j] > 0.0);
  }
  if (!bad && !nonfinite) {
    int nf = 0;
    for (int e = lane; e < N * NX * NX; e += W64) nf |= !isfinite(C.A[e]);
    for (int e = lane; e < N * NX * NU; e += W64) nf |= !isfinite(C.B[e]);
    for (int e = lane; e < N * NX; e += W64) {
      nf |= !isfinite(C.x_ref[e]);
      if (C.e) nf |= !isfinite(C.e[e]);
    }
    if (C.u_ref)
      for (int e = lane; e < N * NU; e += W64) nf |= !isfinite(C.u_ref[e]);
    if (lane < NX) nf |= !isfinite(C.x0[lane]);
    if (p.u_prev && lane < NU) nf |= !isfinite(p.u_prev[(size_t)C.b * NU + lane]);
    nonfinite = wave_max((double)nf) > 0.0;
  }
  const size_t ux = (size_t)C.b * C.n * NU, xx = (size_t)C.b * (C.n + 1) * NX;
  if (bad || nonfinite) {
    for (int e = lane; e < C.n * NU; e += W64) out_u[ux + e] = 0.f;
    for (int e = lane; e < (C.n + 1) * NX; e += W64) out_x[xx + e] = 0.f;
    if (lane == 0) {
      if (out_status) out_status[C.b] = bad ? PINMPC_ST_BADINPUT : PINMPC_ST_NONFINITE;
      if (out_iters) out_iters[C.b] = 0;
    }
    if (out_detail && lane < 4) out_detail[(size_t)C.b * 4 + lane] = 0;
    if (out_res && lane < PINMPC_NRES) out_res[(size_t)C.b * PINMPC_NRES + lane] = __builtin_nanf("");
    return;
  }

  gcf zsrc = (gcf)((accel ? ws.cur : ws.hat) + s0 * NSTATE * NL);
  gcf sf = (gcf)(ws.sf + s0);
  const float tsc = ws.tsc[C.b];
  if (PHASE == 1) admm_point(C, zsrc, sf, tsc);

  double res[PINMPC_NRES] = {0, 0, 0, 0, 0};
  double kkt = 1e300;
  Counts cnt = {0, 0, 0};
  bool ok = false;
  if (refine) {
    // first launch: pass_1 passes (all pass_a when pass_1 is 0); the rest of
    // the passes, the interior point and the polish in the second launch
    const int p1 = (pass_1 > 0 && pass_1 < pass_a) ? pass_1 : pass_a;
    if (PHASE == 1) {
      faces_from_u(C, C.ru, 1e-5);
      bool cycled = false;
      ok = active_set_loop<LONG>(C, sh, p1, tol, &cnt, res, &kkt, &cycled);
      const bool more = !cycled && p1 < pass_a;
      if (!ok && (more || ipm_max > 0)) {
        if (lane == 0) {
          const int slot = atomicAdd(ws.rcount, 1);
          ws.rlist[slot] = C.b;
          // passes (< 2^10, settings are capped at 1000) and stages factored
          // (< 2^20) so far, and whether active-set passes remain
          ws.rpass[C.b] = cnt.eq | (cnt.stf << 10) | (more ? (1 << 30) : 0);
        }
        return;
      }
    } else {
      const int rp = ws.rpass[C.b];
      cnt.eq = rp & 1023;
      cnt.stf = (rp >> 10) & ((1 << 20) - 1);
      if ((rp >> 30) & 1) {
        // resume the active-set passes from the faces the first launch left
        ok = active_set_loop<LONG>(C, sh, pass_a - cnt.eq, tol, &cnt, res, &kkt);
      }
      if (!ok && ipm_max > 0) {
        // interior point from the ADMM point
        admm_point(C, zsrc, sf, tsc);
        rollout_ru(C, sh);
        cnt.ipm = ipm<LONG>(C, sh, ipm_max, tol, &cnt, res, &kkt, &ok);
        if (!ok) ok = active_set_loop<LONG>(C, sh, pass_c, tol, &cnt, res, &kkt);
      }
    }
    // the dynamics residual of the returned trajectory, checked independently
    // of the rollout that produced it
    res[0] = dyn_residual(C);
    ok = ok && res[0] <= tol;
  } else {
    // the ADMM point as it is: rollout, faces from slack, residuals
    faces_from_u(C, C.ru, 1e-5);
    rollout_ru(C, sh);
    const double ts = costates_grad<LONG>(C, sh);
    kkt = multipliers_kkt(C, res, ts);
    res[0] = dyn_residual(C);
  }

  // outputs
  gsync();
  for (int e = lane; e < C.n * NU; e += W64)
    out_u[ux + e] = (e < N * NU) ? (float)C.ru[e] : 0.f;
  for (int e = lane; e < (C.n + 1) * NX; e += W64)
    out_x[xx + e] = (e < (N + 1) * NX) ? (float)C.rx[e] : 0.f;
  if (lane == 0) {
    // the solve's refinement work (stages of every pass and iteration)
    atomicAdd(ws.work, (unsigned long long)(cnt.eq + cnt.ipm) * (unsigned long long)N);
    if (out_status)
      out_status[C.b] = refine ? (ok ? PINMPC_ST_OK : PINMPC_ST_UNPOLISHED) : PINMPC_ST_MAXITER;
    if (out_iters) out_iters[C.b] = admm_iters + cnt.eq + cnt.ipm;
  }
  if (out_detail && lane < 4) {
    const int v = lane == 0 ? cnt.eq : lane == 1 ? cnt.ipm : lane == 2 ? cnt.stf : PHASE;
    out_detail[(size_t)C.b * 4 + lane] = v;
  }
  if (out_res) {
    for (int i = 0; i < PINMPC_NRES; ++i)
      if (lane == i) out_res[(size_t)C.b * PINMPC_NRES + i] = (float)res[i];
  }
}

}  // namespace

size_t scan_lds_bytes(int W) {
  return W > 1 ? (size_t)(W - 1) * sizeof(ShR) + (size_t)W * 4 * TILE_D * sizeof(double) : 0;
}

hipError_t refine_prepare() {
  // the scanning kernels may take more dynamic LDS than the default limit
  const int lds = (int)scan_lds_bytes(SCAN_WMAX);
  const void* k[] = {reinterpret_cast<const void*>(&refine_kernel<1, false, true>),
                     reinterpret_cast<const void*>(&refine_kernel<1, true, true>),
                     reinterpret_cast<const void*>(&refine_kernel<2, false, true>),
                     reinterpret_cast<const void*>(&refine_kernel<2, true, true>)};
  for (const void* f : k) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_refine(const Problem& p, const Workspace& w, const pinmpc_settings& s,
                         const pinmpc_out& out, hipStream_t st) {
  if (p.batch == 0) return hipSuccess;
  const bool second =
      s.refine && (s.ipm_iters > 0 || (s.first_passes > 0 && s.first_passes < s.refine_passes));
  if (second) {
    // the hand-off counter starts at zero (a fill kernel: graph-safe)
    const hipError_t e = launch_fill_i32(w.rcount, 1, 0, 0, st);
    if (e != hipSuccess) return e;
  }
  // the horizon scan: one wave per chunk, dynamic LDS for the helpers'
  // buffers, the summaries and the boundary values
  const int W = s.scan > 1 ? s.scan : 1;
  const size_t lds = scan_lds_bytes(W);
#define PINMPC_REFINE(PH, L, SC)                                                               \
  hipLaunchKernelGGL((refine_kernel<PH, L, SC>), dim3(p.batch), dim3(64 * W), lds, st, p, w,     \
                     out.u, out.x, out.res, out.iters, out.status, out.detail, s.iters, s.accel, \
                     s.refine, s.refine_passes, s.ipm_iters, s.polish_passes, s.kkt_tol,        \
                     s.first_passes)
  // horizons beyond PINMPC_NMAX keep the rollout's and the costates' stage
  // buffers in the scratch block (refine_block_doubles sizes it so)
  const bool lng = p.n_max > PINMPC_NMAX;
  for (int ph = 1; ph <= (second ? 2 : 1); ++ph) {
    if (ph == 1) {
      if (W > 1) {
        if (lng) PINMPC_REFINE(1, true, true);
        else PINMPC_REFINE(1, false, true);
      } else {
        if (lng) PINMPC_REFINE(1, true, false);
        else PINMPC_REFINE(1, false, false);
      }
    } else {
      if (W > 1) {
        if (lng) PINMPC_REFINE(2, true, true);
        else PINMPC_REFINE(2, false, true);
      } else {
        if (lng) PINMPC_REFINE(2, true, false);
        else PINMPC_REFINE(2, false, false);
      }
    }
  }
#undef PINMPC_REFINE
  return hipGetLastError();
}

}  // namespace pinmpc
