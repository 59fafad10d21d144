// Per-stage ADMM setup (Sec. III cached quantities), one 64-lane wave per stage.
//
// For stage k of problem b, with block-constant input scaling S_k
// (force triples m g / stance count, moment triples tau_max):
//   Bt_k = B_k S_k                                  (scaled inputs u = S ut)
//   M_k  = (Bt_k^T Bt_k + I)^{-1}                   (so J_k w = M_k (Bt^T w_x + w_u))
//   H_k  = (Qbar_k + rho I + [k < N-1] rho Abar_{k+1}^T Abar_{k+1})^{-1}
//          Qbar_k = diag(Q, R S_k^2),  Abar^T Abar = [[A^T A, A^T Bt], [Bt^T A, Bt^T Bt + I]]
//   qbar_k = (Q x_ref[k], R S_k u_ref[k])
// FP32 arithmetic throughout (the ADMM that uses these runs in FP32; both
// matrices inverted are symmetric positive definite with eigenvalues >= 1 and
// >= rho, so Gauss-Jordan without pivoting is stable).
#include "pinmpc_internal.h"

namespace pinmpc {

namespace {

__device__ inline int stance_count(const uint8_t* c) { return (c[0] != 0) + (c[1] != 0); }

__device__ inline float scale_of(const Problem& p, int b, int k, int j, bool scaling) {
  if (!scaling) return 1.f;
  const size_t s = (size_t)b * p.n_max + k;
  const int ns = stance_count(p.contact + 2 * s);
  const float sf = weight_of(p, b) / (float)(ns > 0 ? ns : 1);
  return (j % 6) < 3 ? sf : p.tau_max[b];
}

// 1/a from the hardware estimate and one Newton step (SPD pivots: finite and
// positive), within about an ulp of the FP32 quotient.
__device__ inline float recip_f(float a) {
  float r = __builtin_amdgcn_rcpf(a);
  const float e = fmaf(-a, r, 1.f);
  return fmaf(r, e, r);
}

__device__ inline float readlane_f(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

// Gauss-Jordan without pivoting on a system whose column c is held by lane c
// of the wave (col[r] is row r); the pivot column is broadcast from its lane.
// Afterwards a lane holding column c of [M | X] holds column c of
// [I | M^{-1} X].
template <int n>
__device__ inline void gj_columns_f(float (&col)[n]) {
#pragma unroll
  for (int p = 0; p < n; ++p) {
    float pc[n];
#pragma unroll
    for (int r = 0; r < n; ++r) pc[r] = readlane_f(col[r], p);
    const float t = col[p] * recip_f(pc[p]);
#pragma unroll
    for (int r = 0; r < n; ++r)
      if (r != p) col[r] = fmaf(-pc[r], t, col[r]);
    col[p] = t;
  }
}

__global__ void __launch_bounds__(64) setup_kernel(Problem p, Workspace ws, float rho,
                                                   int scaling, int bf16) {
  const int s = blockIdx.x;                    // stage index b * n_max + k
  const int b = s / p.n_max, k = s % p.n_max;
  const int lane = threadIdx.x;
  const int N = horizon(p, b);
  __shared__ float sTop[NX * NL];              // [A_{k+1} | Bt_{k+1}], 13 x 25
  __shared__ float sBt[NX * NU];               // Bt_k
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
    const float v = Bk[i] * scale_of(p, b, k, j, sc);
    sBt[i] = v;
    ws.Bt[(size_t)s * NX * NU + i] = v;
    if (bf16) ws.Btbf[(size_t)s * NX * NU + i] = to_bf16(v);
  }
  const bool has_next = (k + 1 < N);
  if (has_next) {
    const float* A1 = p.A + (size_t)(s + 1) * NX * NX;
    const float* B1 = p.B + (size_t)(s + 1) * NX * NU;
    for (int e = lane; e < NX * NL; e += 64) {
      const int i = e / NL, c = e % NL;
      sTop[e] = (c < NX) ? A1[i * NX + c] : B1[i * NU + c - NX] * scale_of(p, b, k + 1, c - NX, sc);
    }
  }
  if (lane == 0) {
    ws.sf[s] = scale_of(p, b, k, 0, sc);
    if (k == 0) ws.tsc[b] = sc ? p.tau_max[b] : 1.f;
  }
  if (bf16) {
    const float* A = p.A + (size_t)s * NX * NX;
    for (int i = lane; i < NX * NX; i += 64) ws.Abf[(size_t)s * NX * NX + i] = to_bf16(A[i]);
  }
  __syncthreads();

  // H_k^{-1} = diag(Q, R S^2) + rho I + [has_next] rho Abar_{k+1}^T Abar_{k+1},
  // with Abar_{k+1} = [[A, Bt], [0, I]]: lane c < 25 forms its column c,
  // lanes 25..49 hold the identity's columns
  {
    float col[NL];
    if (lane < NL) {
      float top[NX];
#pragma unroll
      for (int i = 0; i < NX; ++i) top[i] = has_next ? sTop[i * NL + lane] : 0.f;
      float dg;
      if (lane < NX) {
        dg = p.Q[(size_t)b * NX + lane];
      } else {
        const float sj = scale_of(p, b, k, lane - NX, sc);
        dg = p.R[(size_t)b * NU + lane - NX] * sj * sj;
      }
#pragma unroll
      for (int r = 0; r < NL; ++r) {
        float g = 0.f;
        if (has_next) {
#pragma unroll
          for (int i = 0; i < NX; ++i) g = fmaf(sTop[i * NL + r], top[i], g);
          if (r >= NX && r == lane) g += 1.f;
        }
        col[r] = rho * g + ((r == lane) ? dg + rho : 0.f);
      }
    } else {
#pragma unroll
      for (int r = 0; r < NL; ++r) col[r] = (r == lane - NL) ? 1.f : 0.f;
    }
    gj_columns_f<NL>(col);
    if (lane >= NL && lane < 2 * NL) {
      const int c = lane - NL;
#pragma unroll
      for (int r = 0; r < NL; ++r) {
        if (r <= c) {
          const float v = col[r];
          ws.Hp[(size_t)s * NH + pk(r, c, NL)] = v;
          if (bf16) ws.Hbf[(size_t)s * NH + pk(r, c, NL)] = to_bf16(v);
        }
      }
    }
  }
  // M_k = (Bt^T Bt + I)^{-1}: lane c < 12 forms column c of Bt^T Bt + I,
  // lanes 12..23 hold the identity's columns
  {
    float col[NU];
    if (lane < NU) {
      float bc[NX];
#pragma unroll
      for (int i = 0; i < NX; ++i) bc[i] = sBt[i * NU + lane];
#pragma unroll
      for (int r = 0; r < NU; ++r) {
        float g = 0.f;
#pragma unroll
        for (int i = 0; i < NX; ++i) g = fmaf(sBt[i * NU + r], bc[i], g);
        col[r] = g + ((r == lane) ? 1.f : 0.f);
      }
    } else {
#pragma unroll
      for (int r = 0; r < NU; ++r) col[r] = (r == lane - NU) ? 1.f : 0.f;
    }
    gj_columns_f<NU>(col);
    if (lane >= NU && lane < 2 * NU) {
      const int c = lane - NU;
#pragma unroll
      for (int r = 0; r < NU; ++r) {
        if (r <= c) {
          const float v = col[r];
          ws.Mp[(size_t)s * NM + pk(r, c, NU)] = v;
          if (bf16) ws.Mbf[(size_t)s * NM + pk(r, c, NU)] = to_bf16(v);
        }
      }
    }
  }
  if (lane < NL) {
    float q;
    if (lane < NX) {
      q = p.Q[(size_t)b * NX + lane] * p.x_ref[(size_t)s * NX + lane];
    } else {
      const int j = lane - NX;
      const float ur = p.u_ref ? p.u_ref[(size_t)s * NU + j] : 0.f;
      q = p.R[(size_t)b * NU + j] * scale_of(p, b, k, j, sc) * ur;
    }
    ws.qb[(size_t)s * NL + lane] = q;
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
