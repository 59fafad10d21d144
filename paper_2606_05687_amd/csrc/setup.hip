// Per-stage ADMM setup (Sec. III cached quantities), one 64-lane wave per stage.
//
// For stage k of problem b, with block-constant input scaling S_k
// (force triples m g / stance count, moment triples tau_max):
//   Bt_k = B_k S_k                                  (scaled inputs u = S ut)
//   M_k  = (Bt_k^T Bt_k + I)^{-1}                   (so J_k w = M_k (Bt^T w_x + w_u))
//   H_k  = (Qbar_k + rho I + [k < N-1] rho Abar_{k+1}^T Abar_{k+1})^{-1}
//          Qbar_k = diag(Q, R S_k^2),  Abar^T Abar = [[A^T A, A^T Bt], [Bt^T A, Bt^T Bt + I]]
//   qbar_k = (Q x_ref[k], R S_k u_ref[k])
// Products and inversions run in FP64 and are stored in FP32.
#include "pinmpc_internal.h"

namespace pinmpc {

namespace {

__device__ inline int stance_count(const uint8_t* c) { return (c[0] != 0) + (c[1] != 0); }

__device__ inline double scale_of(const Problem& p, int b, int k, int j, bool scaling) {
  if (!scaling) return 1.0;
  const size_t s = (size_t)b * p.n_max + k;
  const int ns = stance_count(p.contact + 2 * s);
  const double sf = (double)weight_of(p, b) / (ns > 0 ? ns : 1);
  return (j % 6) < 3 ? sf : (double)p.tau_max[b];
}

// In-place Gauss-Jordan inverse of an SPD n x n matrix held in LDS as the
// augmented [n][2n] array [M | I]; on return the right half is M^{-1}.
// SPD matrices need no pivoting.  n <= 32.
__device__ void gj_inverse(double* aug, int n) {
  __shared__ double fac[32];
  const int lane = threadIdx.x;
  const int w = 2 * n;
  for (int j = 0; j < n; ++j) {
    __syncthreads();
    const double piv = aug[j * w + j];
    __syncthreads();
    for (int c = lane; c < w; c += 64) aug[j * w + c] /= piv;
    __syncthreads();
    if (lane < n) fac[lane] = aug[lane * w + j];
    __syncthreads();
    for (int e = lane; e < n * w; e += 64) {
      const int r = e / w, c = e % w;
      if (r != j) aug[r * w + c] -= fac[r] * aug[j * w + c];
    }
  }
  __syncthreads();
}

__global__ void __launch_bounds__(64) setup_kernel(Problem p, Workspace ws, float rho,
                                                   int scaling, int bf16) {
  const int s = blockIdx.x;                    // stage index b * n_max + k
  const int b = s / p.n_max, k = s % p.n_max;
  const int lane = threadIdx.x;
  const int N = horizon(p, b);
  __shared__ double sA1[NX * NX];              // A_{k+1}
  __shared__ double sBt[NX * NU];              // Bt_k
  __shared__ double sBt1[NX * NU];             // Bt_{k+1}
  __shared__ double augM[NU * 2 * NU];
  __shared__ double augH[NL * 2 * NL];
  const bool sc = scaling != 0;

  if (k >= N) {   // padding stage: benign values, never read by the sweep
    for (int i = lane; i < NX * NU; i += 64) ws.Bt[(size_t)s * NX * NU + i] = 0.f;
    for (int i = lane; i < NH; i += 64) ws.Hp[(size_t)s * NH + i] = 0.f;
    for (int i = lane; i < NM; i += 64) ws.Mp[(size_t)s * NM + i] = 0.f;
    for (int i = lane; i < NL; i += 64) ws.qb[(size_t)s * NL + i] = 0.f;
    if (lane == 0) ws.sf[s] = 1.f;
    return;
  }
  const float* Bk = p.B + (size_t)s * NX * NU;
  for (int i = lane; i < NX * NU; i += 64) {
    const int j = i % NU;
    const double v = (double)Bk[i] * scale_of(p, b, k, j, sc);
    sBt[i] = v;
    ws.Bt[(size_t)s * NX * NU + i] = (float)v;
  }
  const bool has_next = (k + 1 < N);
  if (has_next) {
    const float* A1 = p.A + (size_t)(s + 1) * NX * NX;
    const float* B1 = p.B + (size_t)(s + 1) * NX * NU;
    for (int i = lane; i < NX * NX; i += 64) sA1[i] = (double)A1[i];
    for (int i = lane; i < NX * NU; i += 64) sBt1[i] = (double)B1[i] * scale_of(p, b, k + 1, i % NU, sc);
  }
  if (lane == 0) {
    ws.sf[s] = (float)scale_of(p, b, k, 0, sc);
    if (k == 0) ws.tsc[b] = sc ? p.tau_max[b] : 1.f;
  }
  __syncthreads();

  // M_k: [Bt^T Bt + I | I]
  for (int e = lane; e < NU * NU; e += 64) {
    const int r = e / NU, c = e % NU;
    double acc = (r == c) ? 1.0 : 0.0;
    for (int i = 0; i < NX; ++i) acc += sBt[i * NU + r] * sBt[i * NU + c];
    augM[r * 2 * NU + c] = acc;
    augM[r * 2 * NU + NU + c] = (r == c) ? 1.0 : 0.0;
  }
  // H_k^{-1}: diag(Q, R S^2) + rho I + [has_next] rho Abar_{k+1}^T Abar_{k+1}
  for (int e = lane; e < NL * NL; e += 64) {
    const int r = e / NL, c = e % NL;
    double acc = 0.0;
    if (r == c) {
      if (r < NX) acc = (double)p.Q[(size_t)b * NX + r];
      else {
        const double sj = scale_of(p, b, k, r - NX, sc);
        acc = (double)p.R[(size_t)b * NU + r - NX] * sj * sj;
      }
      acc += rho;
    }
    if (has_next) {
      double g = 0.0;
      // Abar_{k+1} columns: c < 13 -> (A col c; 0), c >= 13 -> (Bt col c-13; e_{c-13})
      for (int i = 0; i < NX; ++i) {
        const double ar = r < NX ? sA1[i * NX + r] : sBt1[i * NU + (r - NX)];
        const double ac = c < NX ? sA1[i * NX + c] : sBt1[i * NU + (c - NX)];
        g += ar * ac;
      }
      if (r >= NX && r == c) g += 1.0;
      acc += rho * g;
    }
    augH[r * 2 * NL + c] = acc;
    augH[r * 2 * NL + NL + c] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  gj_inverse(augM, NU);
  gj_inverse(augH, NL);
  for (int r = 0; r < NU; ++r)
    for (int c = r + lane; c < NU; c += 64)
      ws.Mp[(size_t)s * NM + pk(r, c, NU)] =
          (float)(0.5 * (augM[r * 2 * NU + NU + c] + augM[c * 2 * NU + NU + r]));
  for (int r = 0; r < NL; ++r)
    for (int c = r + lane; c < NL; c += 64)
      ws.Hp[(size_t)s * NH + pk(r, c, NL)] =
          (float)(0.5 * (augH[r * 2 * NL + NL + c] + augH[c * 2 * NL + NL + r]));
  if (bf16) {
    const float* A = p.A + (size_t)s * NX * NX;
    for (int i = lane; i < NX * NX; i += 64) ws.Abf[(size_t)s * NX * NX + i] = to_bf16(A[i]);
    for (int i = lane; i < NX * NU; i += 64)
      ws.Btbf[(size_t)s * NX * NU + i] = to_bf16((float)sBt[i]);
    for (int r = 0; r < NU; ++r)
      for (int c = r + lane; c < NU; c += 64)
        ws.Mbf[(size_t)s * NM + pk(r, c, NU)] = to_bf16(ws.Mp[(size_t)s * NM + pk(r, c, NU)]);
    for (int r = 0; r < NL; ++r)
      for (int c = r + lane; c < NL; c += 64)
        ws.Hbf[(size_t)s * NH + pk(r, c, NL)] = to_bf16(ws.Hp[(size_t)s * NH + pk(r, c, NL)]);
  }
  if (lane < NL) {
    double q;
    if (lane < NX) {
      q = (double)p.Q[(size_t)b * NX + lane] * (double)p.x_ref[(size_t)s * NX + lane];
    } else {
      const int j = lane - NX;
      const double ur = p.u_ref ? (double)p.u_ref[(size_t)s * NU + j] : 0.0;
      q = (double)p.R[(size_t)b * NU + j] * scale_of(p, b, k, j, sc) * ur;
    }
    ws.qb[(size_t)s * NL + lane] = (float)q;
  }
}

}  // namespace

hipError_t launch_setup(const Problem& p, const Workspace& w, const pinmpc_settings& s,
                        hipStream_t st) {
  const size_t stages = (size_t)p.batch * p.n_max;
  if (stages == 0) return hipSuccess;
  hipLaunchKernelGGL(setup_kernel, dim3((unsigned)stages), dim3(64), 0, st, p, w, s.rho,
                     s.scaling, s.precision);
  return hipGetLastError();
}

}  // namespace pinmpc
