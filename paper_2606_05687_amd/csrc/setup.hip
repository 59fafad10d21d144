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

__global__ void __launch_bounds__(64) setup_kernel(Problem p, Workspace ws, float rho,
                                                   int scaling, int bf16) {
  const int s = blockIdx.x;                    // stage index b * n_max + k
  const int b = s / p.n_max, k = s % p.n_max;
  const int lane = threadIdx.x;
  const int N = horizon(p, b);
  __shared__ double sTop[NX * NL];             // [A_{k+1} | Bt_{k+1}], 13 x 25
  __shared__ double sBt[NX * NU];              // Bt_k
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
    if (bf16) ws.Btbf[(size_t)s * NX * NU + i] = to_bf16((float)v);
  }
  const bool has_next = (k + 1 < N);
  if (has_next) {
    const float* A1 = p.A + (size_t)(s + 1) * NX * NX;
    const float* B1 = p.B + (size_t)(s + 1) * NX * NU;
    for (int e = lane; e < NX * NL; e += 64) {
      const int i = e / NL, c = e % NL;
      sTop[e] = (c < NX) ? (double)A1[i * NX + c]
                         : (double)B1[i * NU + c - NX] * scale_of(p, b, k + 1, c - NX, sc);
    }
  }
  if (lane == 0) {
    ws.sf[s] = (float)scale_of(p, b, k, 0, sc);
    if (k == 0) ws.tsc[b] = sc ? p.tau_max[b] : 1.f;
  }
  if (bf16) {
    const float* A = p.A + (size_t)s * NX * NX;
    for (int i = lane; i < NX * NX; i += 64) ws.Abf[(size_t)s * NX * NX + i] = to_bf16(A[i]);
  }
  __syncthreads();

  // H_k^{-1} = diag(Q, R S^2) + rho I + [has_next] rho Abar_{k+1}^T Abar_{k+1},
  // with Abar_{k+1} = [[A, Bt], [0, I]]: lane c < 25 forms its column c
  {
    double col[NL];
    if (lane < NL) {
      double top[NX];
#pragma unroll
      for (int i = 0; i < NX; ++i) top[i] = has_next ? sTop[i * NL + lane] : 0.0;
      double dg;
      if (lane < NX) {
        dg = (double)p.Q[(size_t)b * NX + lane];
      } else {
        const double sj = scale_of(p, b, k, lane - NX, sc);
        dg = (double)p.R[(size_t)b * NU + lane - NX] * sj * sj;
      }
#pragma unroll
      for (int r = 0; r < NL; ++r) {
        double g = 0.0;
        if (has_next) {
#pragma unroll
          for (int i = 0; i < NX; ++i) g += sTop[i * NL + r] * top[i];
          if (r >= NX && r == lane) g += 1.0;
        }
        col[r] = rho * g + ((r == lane) ? dg + rho : 0.0);
      }
    } else {
#pragma unroll
      for (int r = 0; r < NL; ++r) col[r] = (r == lane - NL) ? 1.0 : 0.0;
    }
    gj_columns<NL>(col);
    if (lane >= NL && lane < 2 * NL) {
      const int c = lane - NL;
#pragma unroll
      for (int r = 0; r < NL; ++r) {
        if (r <= c) {
          const float v = (float)col[r];
          ws.Hp[(size_t)s * NH + pk(r, c, NL)] = v;
          if (bf16) ws.Hbf[(size_t)s * NH + pk(r, c, NL)] = to_bf16(v);
        }
      }
    }
  }
  // M_k = (Bt^T Bt + I)^{-1}: Gauss-Jordan on [Bt^T Bt + I | I] with lane
  // 16 R + c holding column c of the matrix (c < 12, the same in every row R)
  // or identity column 4 R + c - 12; pivot columns by DPP row broadcast
  {
    static_assert(NU == 12, "row elimination is written for 12 inputs");
    const int hc = lane & 15, rhs = 4 * (lane >> 4) + hc - NU;
    double col[NU];
    if (hc < NU) {
      double bc[NX];
#pragma unroll
      for (int i = 0; i < NX; ++i) bc[i] = sBt[i * NU + hc];
#pragma unroll
      for (int r = 0; r < NU; ++r) {
        double g = (r == hc) ? 1.0 : 0.0;
#pragma unroll
        for (int i = 0; i < NX; ++i) g += sBt[i * NU + r] * bc[i];
        col[r] = g;
      }
    } else {
#pragma unroll
      for (int r = 0; r < NU; ++r) col[r] = (r == rhs) ? 1.0 : 0.0;
    }
    gj_rows(col);
    if (hc >= NU && rhs < NU) {
      const int c = rhs;
#pragma unroll
      for (int r = 0; r < NU; ++r) {
        if (r <= c) {
          const float v = (float)col[r];
          ws.Mp[(size_t)s * NM + pk(r, c, NU)] = v;
          if (bf16) ws.Mbf[(size_t)s * NM + pk(r, c, NU)] = to_bf16(v);
        }
      }
    }
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
