// Stage matrices A_k, B_k of the centroidal model from compact physics, on the
// device (the paper's discrete centroidal dynamics of Sec. II-A, obtained along
// the planned contact sequence as Sec. III states), in the 13-state single-
// rigid-body form with gravity as a state, forward Euler:
//
//   A_k = I + dt A_c:  [0:3, 6:9] = R_z(psi_k)^T   (angle rates from omega)
//                      [3:6, 9:12] = I             (CoM from velocity)
//                      [11, 12] = 1                (gravity state into v_z)
//   B_k = dt B_c:      [6:9, 6i:6i+3]   = I_w^{-1} [p_{i,k} - c_ref,k]_x
//                      [6:9, 6i+3:6i+6] = I_w^{-1}
//                      [9:12, 6i:6i+3]  = I / m
//   I_w^{-1} = R_z(psi_k) diag(1 / I_body) R_z(psi_k)^T
//
// Model 1, the paper's own 9-state form (CoM c, linear momentum l, angular
// momentum k about the CoM; Sec. II-A) in slots 0..8, slots 9..12 inert:
//
//   A_k: I + [0:3, 3:6] = dt / m I
//   B_k: [3:6, 6i:6i+3] = dt I,  [6:9, 6i:6i+3] = dt [p_{i,k} - c_ref,k]_x,
//        [6:9, 6i+3:6i+6] = dt I
//   e_k: [5] = -dt m 9.81 (gravity on the linear momentum)
//
// FP32 arithmetic.  The kernel is bound by its stores (1300 B per stage
// written, about 60 B read): a block handles STAGES consecutive stages, whose
// A blocks (and B blocks) are contiguous in memory, so consecutive threads
// store consecutive floats; the per-stage quantities (rotation, inverse
// inertia, inverse inertia times the lever-arm cross matrices) are formed once
// per stage into LDS first.
#include "pinmpc_internal.h"

namespace pinmpc {

namespace {

constexpr int STAGES = 16;     // stages per block
constexpr int THREADS = 256;
constexpr int NQ = 32;         // per-stage quantities in LDS

// LDS layout of one stage's quantities:
//   0..8   I_w^{-1} (row-major; model 1: I)
//   9..26  I_w^{-1} [r_i]_x, i = 0, 1 (model 1: [r_i]_x)
//   27 cos(psi)  28 sin(psi)  29 dt  30 dt / m  31 valid (k < N)
// (model 1 keeps m dt 9.81 in 28, its gravity term)
__global__ void __launch_bounds__(THREADS) dynamics_kernel(Physics ph, float* __restrict__ A,
                                                           float* __restrict__ Bm,
                                                           float* __restrict__ E) {
  __shared__ float q[STAGES][NQ];
  const size_t S = (size_t)ph.batch * ph.n_max;
  const size_t s0 = (size_t)blockIdx.x * STAGES;
  const int ns = (int)((S - s0) < (size_t)STAGES ? (S - s0) : (size_t)STAGES);
  const int t = threadIdx.x;
  if (t < ns) {
    const size_t s = s0 + t;
    const int b = (int)(s / ph.n_max), k = (int)(s % ph.n_max);
    const int N = ph.N ? ph.N[b] : ph.n_max;
    float* Q = q[t];
    float c = 1.f, sn = 0.f;
    float W[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f};
    if (ph.model == 0) {
      const float psi = ph.yaw[s];
      c = cosf(psi);
      sn = sinf(psi);
      const float ia = 1.f / ph.inertia[3 * b], ib = 1.f / ph.inertia[3 * b + 1],
                  ic = 1.f / ph.inertia[3 * b + 2];
      // R diag(ia, ib, ic) R^T with R = R_z(psi)
      const float w00 = c * c * ia + sn * sn * ib, w01 = c * sn * (ia - ib);
      const float w11 = sn * sn * ia + c * c * ib;
      W[0] = w00; W[1] = w01; W[3] = w01; W[4] = w11; W[8] = ic;
    }
    for (int j = 0; j < 9; ++j) Q[j] = W[j];
    for (int i = 0; i < NCONTACT; ++i) {
      const float rx = ph.feet[(s * NCONTACT + i) * 3 + 0] - ph.c_ref[s * 3 + 0];
      const float ry = ph.feet[(s * NCONTACT + i) * 3 + 1] - ph.c_ref[s * 3 + 1];
      const float rz = ph.feet[(s * NCONTACT + i) * 3 + 2] - ph.c_ref[s * 3 + 2];
      // [r]_x = [[0, -rz, ry], [rz, 0, -rx], [-ry, rx, 0]]
      const float X[9] = {0.f, -rz, ry, rz, 0.f, -rx, -ry, rx, 0.f};
      for (int r = 0; r < 3; ++r)
        for (int cc = 0; cc < 3; ++cc)
          Q[9 + 9 * i + 3 * r + cc] =
              W[3 * r] * X[cc] + W[3 * r + 1] * X[3 + cc] + W[3 * r + 2] * X[6 + cc];
    }
    const float dt = ph.dt[b];
    Q[27] = c;
    Q[28] = ph.model == 0 ? sn : dt * ph.mass[b] * 9.81f;
    Q[29] = dt;
    Q[30] = dt / ph.mass[b];
    Q[31] = (k < N) ? 1.f : 0.f;
  }
  __syncthreads();
  // A blocks: ns * 169 consecutive floats
  float* Ab = A + s0 * (NX * NX);
  for (int e = t; e < ns * NX * NX; e += THREADS) {
    const int j = e / (NX * NX), rc = e % (NX * NX), r = rc / NX, cc = rc % NX;
    const float* Q = q[j];
    float v = (r == cc) ? 1.f : 0.f;
    if (Q[31] != 0.f && ph.model == 1) {
      if (r < 3 && cc == r + 3) v = Q[30];
    } else if (Q[31] != 0.f) {
      const float dt = Q[29];
      if (r < 3 && cc >= 6 && cc < 9) {
        // R_z^T = [[c, s, 0], [-s, c, 0], [0, 0, 1]]
        const int a = r, bcol = cc - 6;
        float rt = 0.f;
        if (a == 2 && bcol == 2) rt = 1.f;
        else if (a < 2 && bcol < 2) rt = (a == bcol) ? Q[27] : (a == 0 ? Q[28] : -Q[28]);
        v += dt * rt;
      } else if (r >= 3 && r < 6 && cc == r + 6) {
        v += dt;
      } else if (r == 11 && cc == 12) {
        v += dt;
      }
    }
    Ab[e] = v;
  }
  // B blocks: ns * 156 consecutive floats
  float* Bb = Bm + s0 * (NX * NU);
  for (int e = t; e < ns * NX * NU; e += THREADS) {
    const int j = e / (NX * NU), rc = e % (NX * NU), r = rc / NU, cc = rc % NU;
    const float* Q = q[j];
    float v = 0.f;
    if (Q[31] != 0.f && ph.model == 1) {
      const int m = cc % 6, i = cc / 6;
      if (r >= 3 && r < 6 && m < 3 && m == r - 3) v = Q[29];
      else if (r >= 6 && r < 9) v = (m < 3) ? Q[29] * Q[9 + 9 * i + 3 * (r - 6) + m]
                                            : (m - 3 == r - 6 ? Q[29] : 0.f);
    } else if (Q[31] != 0.f) {
      const int i = cc / 6, m = cc % 6;
      if (r >= 6 && r < 9) {
        v = (m < 3) ? Q[29] * Q[9 + 9 * i + 3 * (r - 6) + m] : Q[29] * Q[3 * (r - 6) + (m - 3)];
      } else if (r >= 9 && r < 12 && m < 3 && m == r - 9) {
        v = Q[30];
      }
    }
    Bb[e] = v;
  }
  // affine terms: ns * 13 consecutive floats (model 1: gravity on l_z)
  if (E) {
    float* Eb = E + s0 * NX;
    for (int e = t; e < ns * NX; e += THREADS) {
      const int j = e / NX, r = e % NX;
      const float* Q = q[j];
      Eb[e] = (ph.model == 1 && r == 5 && Q[31] != 0.f) ? -Q[28] : 0.f;
    }
  }
}

}  // namespace

hipError_t launch_dynamics(const Physics& ph, float* A, float* B, float* e, hipStream_t st) {
  const size_t S = (size_t)ph.batch * ph.n_max;
  if (S == 0) return hipSuccess;
  const size_t blocks = (S + STAGES - 1) / STAGES;
  hipLaunchKernelGGL(dynamics_kernel, dim3((unsigned)blocks), dim3(THREADS), 0, st, ph, A, B, e);
  return hipGetLastError();
}

}  // namespace pinmpc
