// Internal definitions shared by the HIP translation units of libpinmpc.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pinmpc.h"

namespace pinmpc {

constexpr int NX = PINMPC_NX;   // 13 states
constexpr int NU = PINMPC_NU;   // 12 inputs
constexpr int NL = NX + NU;     // 25: lifted state (x_k, u_{k-1}) of the velocity form
constexpr int NH = NL * (NL + 1) / 2;   // 325: packed symmetric H_k
constexpr int NM = NU * (NU + 1) / 2;   // 78: packed symmetric M_k
constexpr int NROW = 11;        // wrench rows per stance contact
constexpr int NCONTACT = PINMPC_NCONTACT;   // 2 contacts
constexpr int NSTATE = 5;       // ADMM iterate blocks z, v, theta, beta, lambda

// Dimensions with NC contacts per stage (2: the feet; 4: feet and hands).
template <int NC>
struct Dims {
  static constexpr int U = 6 * NC;                 // inputs
  static constexpr int L = NX + U;                 // lifted state
  static constexpr int H = L * (L + 1) / 2;        // packed symmetric H_k
  static constexpr int M = U * (U + 1) / 2;        // packed symmetric M_k
};
static_assert(Dims<NCONTACT>::L == NL && Dims<NCONTACT>::H == NH && Dims<NCONTACT>::M == NM,
              "two contacts are the default dimensions");

// BF16 (bfloat16) storage: round to nearest even from FP32, and back.
__host__ __device__ inline uint16_t to_bf16(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 1u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float from_bf16(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}

// Operator loads of the sweep kernels: FP32 arrays, or their BF16 copies.
template <bool BF16>
struct OpLoad;
template <>
struct OpLoad<false> {
  const float *A, *Bt, *H, *M;
  __device__ float a(size_t i) const { return A[i]; }
  __device__ float bt(size_t i) const { return Bt[i]; }
  __device__ float h(size_t i) const { return H[i]; }
  __device__ float m(size_t i) const { return M[i]; }
};
template <>
struct OpLoad<true> {
  const uint16_t *A, *Bt, *H, *M;
  __device__ float a(size_t i) const { return from_bf16(A[i]); }
  __device__ float bt(size_t i) const { return from_bf16(Bt[i]); }
  __device__ float h(size_t i) const { return from_bf16(H[i]); }
  __device__ float m(size_t i) const { return from_bf16(M[i]); }
};

// Packed upper-triangular index of symmetric (r, c), n x n.
__host__ __device__ inline int pk(int r, int c, int n) {
  if (r > c) { int t = r; r = c; c = t; }
  return r * n - (r * (r - 1)) / 2 + (c - r);
}

// Problem data as the kernels see it (device pointers; optional ones may be
// null and then mean zero / the documented default).
struct Problem {
  int32_t batch, n_max;
  int32_t nc;   // contacts per stage: 2 or 4 (inputs 6 nc)
  const int32_t* N;
  const float *A, *B, *e, *x0, *u_prev, *x_ref, *u_ref, *Q, *R;
  const uint8_t* contact;
  const float *mu, *fz_max, *tau_max, *weight;
};

// Horizon of problem b clamped to [0, n_max], so that no kernel indexes past
// its problem's stages whatever the caller passed (the refinement flags an
// out-of-range horizon as bad input from the raw value).
__device__ inline int horizon(const Problem& p, int b) {
  if (!p.N) return p.n_max;
  const int N = p.N[b];
  return N < 0 ? 0 : (N > p.n_max ? p.n_max : N);
}
__device__ inline int horizon_raw(const Problem& p, int b) {
  return p.N ? p.N[b] : p.n_max;
}
__device__ inline float weight_of(const Problem& p, int b) {
  return p.weight ? p.weight[b] : 0.5f * p.fz_max[b];
}

// Workspace carved from one device allocation.
struct Workspace {
  // FP32 ADMM operators, per stage s = b * n_max + k
  float* Bt;        // [s][13][12] scaled input matrix B_k S_k
  float* Hp;        // [s][325] packed H_k
  float* Mp;        // [s][78] packed M_k = (Bt^T Bt + I)^{-1}
  float* qb;        // [s][25] linear cost term (Q r_k, Rt ut_ref)
  // BF16 copies of the operators (precision = 1)
  uint16_t* Abf;    // [s][13][13]
  uint16_t* Btbf;   // [s][13][12]
  uint16_t* Hbf;    // [s][325]
  uint16_t* Mbf;    // [s][78]
  float* sf;        // [s] force scale of stage k
  float* tsc;       // [b] moment scale (tau_max, or 1 without scaling)
  // ADMM iterates [s][5][25]: current and extrapolated ("hat")
  float* cur;
  float* hat;
  float* alpha;     // [b] acceleration sequence
  float* cprev;     // [b] restart test value
  int32_t* restarts;// [b]
  uint32_t* flags;  // [b] bit0: nonfinite input, bit1: bad bounds
  // FP64 refinement scratch: one contiguous block per problem
  // (refine_block_doubles(n_max) doubles each), see refine.hip
  double* rblk;
  int32_t* faces;   // [s][2] face code per contact
  int32_t* order;   // [3][b] problems of each horizon class (packing)
  int32_t* counts;  // [4] problems per class
  // refinement hand-off: problems the active-set passes did not certify
  // (second launch: interior point and polish), their count, and the passes
  // each used in the first launch
  int32_t* rlist;   // [b]
  int32_t* rcount;  // [1]
  int32_t* rpass;   // [b]
  // refinement work of the solve: stages of every equality-constrained pass
  // and interior-point iteration, summed over problems (64-bit counter)
  unsigned long long* work;
  // horizon split across workgroups (admm_split.hip): per-stage exchange of
  // one sweep, the sweep's new iterates, the restart-test terms and decisions
  float* sp_aty;    // [s][25] Abar_k^T y_k
  float* sp_du;     // [s][12] du_k
  float* sp_xi;     // [s][25] xi_{k+1}
  float* sp_new;    // [s][5][25] new iterates of the sweep
  float* sp_ct;     // [s] restart-test term of the stage
  float* sp_dec;    // [b][2] extrapolation factor, restart flag
  size_t bytes;
  // warm start (serving): per problem slot index into a device store of
  // iterates [slot][PINMPC_NMAX][5][25]; null / negative index = cold start
  const int32_t* warm_idx;
  float* warm_store;
};

// FP64 scratch of the refinement per problem with n stages.  The stage
// blocks come first, each stored compactly (only the entries that can be
// nonzero; the register tiles are rebuilt from them entry by entry):
//   T    stage input: per contact its 6 x 6 diagonal block (row-major), then
//        its 6 offsets (face projector and point, or the interior-point input
//        Hessian and linear term)
//   K    gains, 12 x 13 row-major
//   L    inverse input Hessian, 12 x 12 row-major (interior-point steps)
//   Hwx  12 x 13 row-major (interior-point steps)
//   S    value function: lower triangle of S (13 x 13, row by row), then s
// Then per stage: feedforward (12), inputs (12), costates (13), gradient (12),
// row multipliers, slacks, interior-point multipliers and their steps
// (5 x 22) and step du (12); and states x and dx ((n+1) x 13 each).
// Horizons beyond PINMPC_NMAX (the long-horizon path) keep two more 16-wide
// per-stage vectors there (the costate chain's and the rollout's stage
// buffers, which live in LDS for shorter horizons).
constexpr int TS_T = 2 * (36 + 6);
constexpr int TS_K = NU * NX;
constexpr int TS_L = NU * NU;
constexpr int TS_H = NU * NX;
constexpr int TS_S = NX * (NX + 1) / 2 + NX;
__host__ __device__ constexpr size_t refine_block_doubles(int n) {
  return (((size_t)n * (TS_T + TS_K + TS_L + TS_H + TS_S + NU + NU + NX + NU + 5 * 2 * NROW + NU) +
           2 * (size_t)(n + 1) * NX + (n > PINMPC_NMAX ? (size_t)n * 32 : 0)) + 3) & ~(size_t)3;
}

// FP64 scratch of the four-contact refinement (refine_wide.hip) per problem
// with n stages: gains (24 x 13), feedforward, inputs, their step and the
// costates (24 each), the stage input terms (per contact a 6 x 6 block and
// six entries), slacks, multipliers, their steps and the complementarity
// target (11 per contact each), the inverse input Hessian (24 x 24) and Hwx
// (24 x 13), then x and dx ((n+1) x 13 each).
__host__ __device__ constexpr size_t refine_wide_block_doubles(int n) {
  return ((size_t)n * (24 * NX + 4 * 24 + 4 * 42 + 5 * 4 * NROW + 24 * 24 + 24 * NX) +
          2 * (size_t)(n + 1) * NX + 3) & ~(size_t)3;
}

// 1/a from the hardware estimate refined by two Newton steps (the pivots of
// SPD eliminations: finite and positive); within about an ulp of the quotient.
__device__ inline double recip(double a) {
  double r = __builtin_amdgcn_rcp(a);
  double e = fma(-a, r, 1.0);
  r = fma(r, e, r);
  e = fma(-a, r, 1.0);
  return fma(r, e, r);
}

__device__ inline double readlane_d(double v, int l) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Gauss-Jordan elimination without pivoting (SPD systems) on a matrix whose
// column c is held in registers by lane c of a 64-lane wave: col[r] is row r.
// The pivot column is broadcast from its lane with readlane (a broadcast
// through LDS was slower: each pivot then waits for an LDS round trip).
// Afterwards each lane holds its column of M^{-1} [rest] where M is the
// leading n x n block (lanes 0..n-1 end with the identity).  Bit p of the
// wave-uniform `unit` marks a pivot whose row and column of the whole system
// are exactly the unit vector e_p: its elimination step changes nothing and
// is skipped (bitwise the same result).
template <int n>
__device__ inline void gj_columns(double (&col)[n], uint32_t unit = 0) {
#pragma unroll
  for (int p = 0; p < n; ++p) {
    if ((unit >> p) & 1u) continue;
    double pc[n];
#pragma unroll
    for (int r = 0; r < n; ++r) pc[r] = readlane_d(col[r], p);
    const double t = col[p] * recip(pc[p]);
#pragma unroll
    for (int r = 0; r < n; ++r)
      if (r != p) col[r] -= pc[r] * t;
    col[p] = t;
  }
}

// Lane P of each 16-lane row of the wave, to every lane of that row (a DPP
// row broadcast of the 64-bit value).
template <int P>
__device__ inline double row_bcast(double v) {
  return __builtin_amdgcn_update_dpp(v, v, 0x150 + P, 0xF, 0xF, true);
}

// c[r] += (c[r] of lane P of this 16-lane row) * s for r = 0..11, as one
// block of DPP fused multiply-adds.  Each instruction reads its own register
// from lane P before writing it, so every lane sees lane P's values from
// before the block.  The leading two wait states separate the block's DPP
// reads from a vector write just before it.
template <int P>
__device__ inline void fmac_row_bcast12(double (&c)[12], double s) {
#define PINMPC_FMAC(i) \
  "v_fmac_f64_dpp %" #i ", %" #i ", %12 row_newbcast:%13 row_mask:0xf bank_mask:0xf bound_ctrl:1\n"
  asm volatile("s_nop 1\n" PINMPC_FMAC(0) PINMPC_FMAC(1) PINMPC_FMAC(2) PINMPC_FMAC(3)
               PINMPC_FMAC(4) PINMPC_FMAC(5) PINMPC_FMAC(6) PINMPC_FMAC(7) PINMPC_FMAC(8)
               PINMPC_FMAC(9) PINMPC_FMAC(10) PINMPC_FMAC(11)
               : "+v"(c[0]), "+v"(c[1]), "+v"(c[2]), "+v"(c[3]), "+v"(c[4]), "+v"(c[5]),
                 "+v"(c[6]), "+v"(c[7]), "+v"(c[8]), "+v"(c[9]), "+v"(c[10]), "+v"(c[11])
               : "v"(s), "i"(P));
#undef PINMPC_FMAC
}

// The same elimination as gj_columns (the same roundings in the same order),
// for a 12-row system whose leading 12 x 12 block sits in lanes 0..11 of
// every 16-lane row of the wave (column c in lane c of each row, the rows
// identical) and whose other columns occupy the remaining lanes of the rows:
// the pivot column reaches its row's lanes through the DPP row broadcast of
// the update instructions themselves.
template <int p = 0>
__device__ inline void gj_rows(double (&col)[12], uint32_t unit = 0) {
  if constexpr (p < 12) {
    if (!((unit >> p) & 1u)) {
      const double t = col[p] * recip(row_bcast<p>(col[p]));
      fmac_row_bcast12<p>(col, -t);   // col[r] - pc[r] t; col[p] is replaced next
      col[p] = t;
    }
    gj_rows<p + 1>(col, unit);
  }
}

// gj_rows on two systems with the same leading block (so the same pivots):
// one reciprocal per pivot, two independent update blocks.
template <int p = 0>
__device__ inline void gj_rows2(double (&a)[12], double (&b)[12], uint32_t unit = 0) {
  if constexpr (p < 12) {
    if (!((unit >> p) & 1u)) {
      const double rp = recip(row_bcast<p>(a[p]));
      const double ta = a[p] * rp, tb = b[p] * rp;
      fmac_row_bcast12<p>(a, -ta);
      fmac_row_bcast12<p>(b, -tb);
      a[p] = ta;
      b[p] = tb;
    }
    gj_rows2<p + 1>(a, b, unit);
  }
}

// Face code of one contact: bits 0..4 force rows active
//   (0: f_x - mu f_z <= 0, 1: -f_x - mu f_z <= 0, 2: f_y - mu f_z <= 0,
//    3: -f_y - mu f_z <= 0, 4: f_z <= fz_max),
// bits 8..13 moment rows (8+a: tau_a <= tau_max, 11+a: -tau_a <= tau_max).
// Rows {0,1} or {2,3} together mean the apex f = 0 (code force bits = 15).
constexpr int FACE_APEX = 15;

// Euclidean projection of y onto {|f_x|,|f_y| <= mu f_z, f_z <= F}
// (candidate enumeration over the faces of the truncated pyramid; the set
// is symmetric in the signs of f_x, f_y, so work on (|y_x|, |y_y|, y_z)).
template <typename T>
__device__ inline void project_pyramid(T mu, T F, T yx, T yy, T yz, T* px, T* py,
                                       T* pz) {
  const T sx = yx < T(0) ? T(-1) : T(1);
  const T sy = yy < T(0) ? T(-1) : T(1);
  const T a = yx * sx, b = yy * sy, z = yz;
  const T tol = T(1e-6) * (T(1) + F);
  T best = T(3.0e38), ba = 0, bb = 0, bz = 0;
  auto consider = [&](T ca, T cb, T cz) {
    if (ca < -tol || cb < -tol || ca > mu * cz + tol || cb > mu * cz + tol || cz > F + tol)
      return;
    const T d = (ca - a) * (ca - a) + (cb - b) * (cb - b) + (cz - z) * (cz - z);
    if (d < best) { best = d; ba = ca; bb = cb; bz = cz; }
  };
  consider(a, b, z);                                   // interior
  const T m2 = T(1) + mu * mu;
  {  // side a = mu z
    const T t = (a - mu * z) / m2;
    consider(a - t, b, z + mu * t);
  }
  {  // side b = mu z
    const T t = (b - mu * z) / m2;
    consider(a, b - t, z + mu * t);
  }
  {  // lateral edge a = b = mu z
    const T t = (mu * a + mu * b + z) / (T(2) * mu * mu + T(1));
    consider(mu * t, mu * t, t);
  }
  consider(a, b, F);                                   // top
  consider(mu * F, b, F);                              // top edge a = mu F
  consider(a, mu * F, F);                              // top edge b = mu F
  consider(mu * F, mu * F, F);                         // top corner
  consider(T(0), T(0), T(0));                          // apex
  *px = sx * ba;
  *py = sy * bb;
  *pz = bz;
}

// Sum of one value per (stage k < N, lifted row r < W) held in LDS at
// cp[k * W + r] (W = 25 with two contacts), in an order fixed by N alone (rows in order within a
// stage, then stages in order), so the result does not depend on the launch
// shape and a problem computes bitwise the same alone or inside any batch.
// ss: N + 1 floats of LDS scratch; t: the calling thread's index among the
// problem's threads (at least N of them).  Every thread of the workgroup must
// call it.
template <int W = NL>
__device__ inline float stage_ordered_sum(const float* cp, float* ss, int N, int t) {
  __syncthreads();
  if (t < N) {
    float a = 0.f;
    for (int r = 0; r < W; ++r) a += cp[t * W + r];
    ss[t] = a;
  }
  __syncthreads();
  if (t == 0) {
    float a = 0.f;
    for (int k = 0; k < N; ++k) a += ss[k];
    ss[N] = a;
  }
  __syncthreads();
  const float v = ss[N];
  __syncthreads();
  return v;
}

// Solve on a given stream, optionally warm-started from (and saving into) a
// device store of iterates (the serving loop uses this; pinmpc_solve passes
// null).  Defined in api.cpp.
int solve_internal(pinmpc_ctx c, const pinmpc_batch* in, const pinmpc_out* out,
                   hipStream_t st, const int32_t* warm_idx, float* warm_store);

// Eager solve (no graph) whose workspace is carved from caller-provided device
// memory `base` of `capacity` bytes; PINMPC_ETOOBIG when the batch needs more.
// Allocates nothing.  Defined in api.cpp.
int solve_in_buffer(pinmpc_ctx c, const pinmpc_batch* in, const pinmpc_out* out,
                    hipStream_t st, void* base, size_t capacity);

// The HIP device a context solves on (-1 for a null context).
int context_device(pinmpc_ctx c);

// Allocate the context's workspace for batch x n ahead of the first solve.
int reserve_internal(pinmpc_ctx c, int32_t batch, int32_t n);

// Host-side pieces of a solve shared by the entry points (api.cpp): carve the
// workspace for batch x n out of `base` (or only size it when base is null;
// returns the bytes), validate settings and a batch, view a batch as the
// kernels' Problem, and enqueue the ADMM sweeps in the form the settings ask
// for.
size_t carve_workspace(char* base, int32_t batch, int32_t n, Workspace* w, int nc = NCONTACT);
int check_settings(const pinmpc_settings* s);
int check_batch(const pinmpc_batch* in);
int contacts_of(const pinmpc_batch* in);   // 2 or 4
Problem to_problem(const pinmpc_batch* in);
int launch_admm_phase(const pinmpc_settings& s, const Problem& p, const Workspace& w, int iters,
                      hipStream_t st);

// Compact physics of the stage matrices (device pointers, see pinmpc_physics).
struct Physics {
  int32_t batch, n_max, model;
  const int32_t* N;
  const float *yaw, *c_ref, *feet, *mass, *inertia, *dt;
};

// Landmark store (see pinmpc_landmarks).
struct LandmarkStore {
  int32_t envs, n_landmarks, ring, ticks_per_step;
  float* com;
  int32_t* tag;
};

// One array of one request to gather into (or scatter from) a serving lane's
// staging: `rows` rows of `row_bytes`, source rows `src_pitch` apart,
// destination rows `dst_pitch` apart; work items (rows) of all descriptors of
// a table are numbered consecutively from `row0`.
enum { COPY_WORDS = 0, COPY_BYTES = 1, COPY_FILL = 2, COPY_HALF = 3 };
struct CopyDesc {
  const void* src;          // null for COPY_FILL
  void* dst;
  uint32_t row_bytes, src_pitch, dst_pitch, rows;
  int32_t op, a, b, pad;    // COPY_FILL writes the int32 pattern a + b i
  uint64_t row0;
};

// Kernel launchers (defined in the .hip units).
hipError_t launch_copy_batch(const CopyDesc* table, int nd, uint64_t rows_total, hipStream_t st);
hipError_t launch_landmarks_clear(const LandmarkStore& st, const uint8_t* mask, hipStream_t s);
hipError_t launch_landmarks_push(const LandmarkStore& st, int n_max, const int32_t* N,
                                 const float* x, int32_t tick, hipStream_t s);
hipError_t launch_landmark_reward(const LandmarkStore& st, const float* com, int32_t tick,
                                  const float* alpha, const float* qc, float sigma,
                                  float* reward, int32_t* used, hipStream_t s);
hipError_t launch_dynamics(const Physics& ph, float* A, float* B, float* e, hipStream_t st);
hipError_t launch_setup(const Problem& p, const Workspace& w, const pinmpc_settings& s,
                        hipStream_t st);
hipError_t launch_admm_init(const Problem& p, const Workspace& w, hipStream_t st);
hipError_t launch_warm_save(const Problem& p, const Workspace& w, int accel, hipStream_t st);
hipError_t launch_fill_i32(int32_t* dst, size_t n, int32_t base, int32_t step, hipStream_t st);
// `sweeps` ADMM sweeps in one launch of the streaming sweep kernel (1: the
// plain form, one launch per sweep; more: iterates resident in registers
// across the sweeps, operators streamed every sweep).
hipError_t launch_admm_sweep(const Problem& p, const Workspace& w, const pinmpc_settings& s,
                             int sweeps, hipStream_t st);
hipError_t launch_admm_fused(const Problem& p, const Workspace& w, const pinmpc_settings& s,
                             int iters, hipStream_t st);
// All sweeps with the horizon split across workgroups (a chain of
// stage-parallel launches per sweep); any horizon up to PINMPC_NMAX_LONG.
hipError_t launch_admm_split(const Problem& p, const Workspace& w, const pinmpc_settings& s,
                             int iters, hipStream_t st);
// Horizon-class packing: class 0 N <= 20, class 1 20 < N <= 40, class 2 N > 40.
constexpr int CLASS_N[3] = {20, 40, PINMPC_NMAX};
static_assert(PINMPC_NMAX_LONG >= PINMPC_NMAX, "long horizons extend the short ones");
hipError_t launch_classify(const Problem& p, const Workspace& w, hipStream_t st);
hipError_t launch_admm_fused_class(const Problem& p, const Workspace& w, const pinmpc_settings& s,
                                   int iters, int cls, hipStream_t st);
hipError_t launch_admm_sweep_class(const Problem& p, const Workspace& w,
                                   const pinmpc_settings& s, int cls, int sweeps,
                                   hipStream_t st);
hipError_t launch_admm_extract(const Problem& p, const Workspace& w, int accel,
                               float* z_out, hipStream_t st);
// Once per device before the first solve: lets the refinement's scanning
// kernels take the dynamic LDS they need (see the scan setting).
hipError_t refine_prepare();
hipError_t launch_refine(const Problem& p, const Workspace& w, const pinmpc_settings& s,
                         const pinmpc_out& out, hipStream_t st);
// The FP64 refinement of problems with four contacts per stage (refine_wide.hip).
hipError_t launch_refine_wide(const Problem& p, const Workspace& w, const pinmpc_settings& s,
                              const pinmpc_out& out, hipStream_t st);


}  // namespace pinmpc
