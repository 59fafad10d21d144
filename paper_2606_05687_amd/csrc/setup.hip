// Per-stage ADMM setup (Sec. III cached quantities), one workgroup per stage.
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

template <int NC>
__device__ inline int stance_count(const uint8_t* c) {
  int n = 0;
#pragma unroll
  for (int i = 0; i < NC; ++i) n += (c[i] != 0);
  return n;
}

template <int NC>
__device__ inline float scale_of(const Problem& p, int b, int k, int j, bool scaling) {
  if (!scaling) return 1.f;
  const size_t s = (size_t)b * p.n_max + k;
  const int ns = stance_count<NC>(p.contact + NC * s);
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

// One workgroup per stage.  With NC = 4 the lifted system has 37 columns and
// [H | I] 74, more than a wave has lanes: the workgroup then holds two waves,
// each eliminating all of H (the same arithmetic in the same order) beside
// its own share of the identity's columns.
template <int NC>
__global__ void __launch_bounds__(64 * (NC / 2)) setup_kernel(Problem p, Workspace ws, float rho,
                                                              int scaling, int bf16) {
  using D = Dims<NC>;
  constexpr int U = D::U, L = D::L;
  const int s = blockIdx.x;                    // stage index b * n_max + k
  const int b = s / p.n_max, k = s % p.n_max;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int N = horizon(p, b);
  __shared__ float sTop[NX * L];               // [A_{k+1} | Bt_{k+1}], 13 x L
  __shared__ float sBt[NX * U];                // Bt_k
  const bool sc = scaling != 0;

  if (k >= N) {   // padding stage: benign values, never read by the sweep
    for (int i = tid; i < NX * U; i += blockDim.x) ws.Bt[(size_t)s * NX * U + i] = 0.f;
    for (int i = tid; i < D::H; i += blockDim.x) ws.Hp[(size_t)s * D::H + i] = 0.f;
    for (int i = tid; i < D::M; i += blockDim.x) ws.Mp[(size_t)s * D::M + i] = 0.f;
    for (int i = tid; i < L; i += blockDim.x) ws.qb[(size_t)s * L + i] = 0.f;
    if (tid == 0) ws.sf[s] = 1.f;
    return;
  }
  // the stage's force and moment scales, and the next stage's (read once:
  // each needs the stage's contact flags and the problem's bounds)
  const float sfk = scale_of<NC>(p, b, k, 0, sc), smk = scale_of<NC>(p, b, k, 3, sc);
  const bool has_next = (k + 1 < N);
  const float sf1 = has_next ? scale_of<NC>(p, b, k + 1, 0, sc) : 1.f;
  const float sm1 = has_next ? scale_of<NC>(p, b, k + 1, 3, sc) : 1.f;
  auto scale_k = [&](int j) { return (j % 6) < 3 ? sfk : smk; };
  const float* Bk = p.B + (size_t)s * NX * U;
  for (int i = tid; i < NX * U; i += blockDim.x) {
    const int j = i % U;
    const float v = Bk[i] * scale_k(j);
    sBt[i] = v;
    ws.Bt[(size_t)s * NX * U + i] = v;
    if (bf16) ws.Btbf[(size_t)s * NX * U + i] = to_bf16(v);
  }
  if (has_next) {
    const float* A1 = p.A + (size_t)(s + 1) * NX * NX;
    const float* B1 = p.B + (size_t)(s + 1) * NX * U;
    for (int e = tid; e < NX * L; e += blockDim.x) {
      const int i = e / L, c = e % L;
      sTop[e] = (c < NX) ? A1[i * NX + c]
                         : B1[i * U + c - NX] * ((c - NX) % 6 < 3 ? sf1 : sm1);
    }
  }
  if (tid == 0) {
    ws.sf[s] = sfk;
    if (k == 0) ws.tsc[b] = sc ? p.tau_max[b] : 1.f;
  }
  if (bf16) {
    const float* A = p.A + (size_t)s * NX * NX;
    for (int i = tid; i < NX * NX; i += blockDim.x) ws.Abf[(size_t)s * NX * NX + i] = to_bf16(A[i]);
  }
  __syncthreads();

  // H_k^{-1} = diag(Q, R S^2) + rho I + [has_next] rho Abar_{k+1}^T Abar_{k+1},
  // with Abar_{k+1} = [[A, Bt], [0, I]]: lane c < L forms its column c, the
  // other lanes of wave w hold the identity's columns w (64 - L) + lane - L
  {
    constexpr int PER = 64 - L;                // identity columns per wave
    const int ic = wave * PER + lane - L;      // this lane's identity column
    float col[L];
    if (lane < L) {
      float top[NX];
#pragma unroll
      for (int i = 0; i < NX; ++i) top[i] = has_next ? sTop[i * L + lane] : 0.f;
      float dg;
      if (lane < NX) {
        dg = p.Q[(size_t)b * NX + lane];
      } else {
        const float sj = scale_k(lane - NX);
        dg = p.R[(size_t)b * U + lane - NX] * sj * sj;
      }
#pragma unroll
      for (int r = 0; r < L; ++r) {
        float g = 0.f;
        if (has_next) {
#pragma unroll
          for (int i = 0; i < NX; ++i) g = fmaf(sTop[i * L + r], top[i], g);
          if (r >= NX && r == lane) g += 1.f;
        }
        col[r] = rho * g + ((r == lane) ? dg + rho : 0.f);
      }
    } else {
#pragma unroll
      for (int r = 0; r < L; ++r) col[r] = (r == ic) ? 1.f : 0.f;
    }
    gj_columns_f<L>(col);
    if (lane >= L && ic < L) {
      const int c = ic;
#pragma unroll
      for (int r = 0; r < L; ++r) {
        if (r <= c) {
          const float v = col[r];
          ws.Hp[(size_t)s * D::H + pk(r, c, L)] = v;
          if (bf16) ws.Hbf[(size_t)s * D::H + pk(r, c, L)] = to_bf16(v);
        }
      }
    }
  }
  if (wave != 0) return;
  // M_k = (Bt^T Bt + I)^{-1}: lane c < U forms column c of Bt^T Bt + I,
  // lanes U..2U-1 hold the identity's columns
  {
    float col[U];
    if (lane < U) {
      float bc[NX];
#pragma unroll
      for (int i = 0; i < NX; ++i) bc[i] = sBt[i * U + lane];
#pragma unroll
      for (int r = 0; r < U; ++r) {
        float g = 0.f;
#pragma unroll
        for (int i = 0; i < NX; ++i) g = fmaf(sBt[i * U + r], bc[i], g);
        col[r] = g + ((r == lane) ? 1.f : 0.f);
      }
    } else {
#pragma unroll
      for (int r = 0; r < U; ++r) col[r] = (r == lane - U) ? 1.f : 0.f;
    }
    gj_columns_f<U>(col);
    if (lane >= U && lane < 2 * U) {
      const int c = lane - U;
#pragma unroll
      for (int r = 0; r < U; ++r) {
        if (r <= c) {
          const float v = col[r];
          ws.Mp[(size_t)s * D::M + pk(r, c, U)] = v;
          if (bf16) ws.Mbf[(size_t)s * D::M + pk(r, c, U)] = to_bf16(v);
        }
      }
    }
  }
  if (lane < L) {
    float q;
    if (lane < NX) {
      q = p.Q[(size_t)b * NX + lane] * p.x_ref[(size_t)s * NX + lane];
    } else {
      const int j = lane - NX;
      const float ur = p.u_ref ? p.u_ref[(size_t)s * U + j] : 0.f;
      q = p.R[(size_t)b * U + j] * scale_k(j) * ur;
    }
    ws.qb[(size_t)s * L + lane] = q;
  }
}

static_assert(2 * Dims<2>::U <= 64 && 2 * Dims<4>::U <= 64, "[M | I] fits one wave");
static_assert(2 * (64 - Dims<4>::L) >= Dims<4>::L && 64 - Dims<2>::L >= Dims<2>::L,
              "the identity columns of [H | I] fit the workgroup's waves");

}  // namespace

hipError_t launch_setup(const Problem& p, const Workspace& w, const pinmpc_settings& s,
                        hipStream_t st) {
  const size_t stages = (size_t)p.batch * p.n_max;
  if (stages == 0) return hipSuccess;
  if (p.nc == 4)
    hipLaunchKernelGGL(setup_kernel<4>, dim3((unsigned)stages), dim3(128), 0, st, p, w, s.rho,
                       s.scaling, s.precision);
  else
    hipLaunchKernelGGL(setup_kernel<2>, dim3((unsigned)stages), dim3(64), 0, st, p, w, s.rho,
                       s.scaling, s.precision);
  return hipGetLastError();
}

}  // namespace pinmpc
