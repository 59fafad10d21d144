// Fused form of the parallel-in-horizon ADMM (Sec. III): all sweeps of a
// problem in one launch, with every thread's share of the stage operators
// loaded once into registers and kept there across the sweeps.
//
// A workgroup owns PPW problems (one, or two or four short ones packed into one
// workgroup), each with its own group of threads and LDS buffers; thread
// (k, r) of a problem's group owns lifted row r of stage k:
//   r < 13 : row r of H_k, row r and column r of A_k, row r of Bt_k
//   r >= 13: row r of H_k, column j = r-13 of Bt_k, row j of M_k
// which is exactly what its share of the stage products needs:
//   (Abar^T y)_r, (Bt^T w)_j, (M t)_j, (H htilde)_r, (Abar xi)_r, (Bbar du)_r.
// Vectors that a product needs whole (w, y, t, htilde, xi_k of the
// neighbour stage, du) are exchanged through LDS; the iterates stay in
// registers and are written back once at the end.  HBM traffic per solve is
// the operators once plus the iterates once, independent of the sweep count.
#include "pinmpc_internal.h"

// Every multiply-add below is either an explicit fmaf or a separate multiply
// and add: no compiler contraction, so every instantiation of the sweep
// (plain or fused, any block size) computes bitwise the same iterates.
#pragma clang fp contract(off)

namespace pinmpc {

namespace {

constexpr int V25 = 25;

// LDS floats of one problem for a capacity of n stages.
__host__ __device__ inline size_t fused_lds_floats(int n) {
  return (size_t)(5 * n * V25 + 4 * n * NU + 32);
}

template <int MAXT, bool BF16, int PPW>
__global__ void __launch_bounds__(MAXT) admm_fused_kernel(Problem p, Workspace ws, float rho,
                                                          int accel, float eta, int iters,
                                                          const int32_t* order,
                                                          const int32_t* count, int lds_n) {
  OpLoad<BF16> op;
  if constexpr (BF16) {
    op.A = ws.Abf; op.Bt = ws.Btbf; op.H = ws.Hbf; op.M = ws.Mbf;
  } else {
    op.A = p.A; op.Bt = ws.Bt; op.H = ws.Hp; op.M = ws.Mp;
  }
  extern __shared__ float lds[];
  const int slots = count ? *count : p.batch;   // problems this launch walks
  if ((int)blockIdx.x * PPW >= slots) return;   // the whole workgroup: uniform
  // this thread's problem slot in the workgroup, and its index in that group
  const int tpp = PPW == 1 ? (int)blockDim.x : (int)blockDim.x / PPW;
  const int sub = PPW == 1 ? 0 : (int)threadIdx.x / tpp;
  const int slot = (int)blockIdx.x * PPW + sub;
  const int n = p.n_max;          // stage stride of the global arrays
  const int ln = lds_n;           // stage capacity of the LDS buffers
  // a slot past the end, or a horizon beyond the LDS capacity (never for a
  // valid packing), leaves its group idle: it still takes part in the barriers
  bool live = slot < slots;
  const int b = live ? (order ? order[slot] : slot) : 0;
  int N = live ? horizon(p, b) : 0;
  if constexpr (PPW == 1) {
    if (N > ln || N == 0) return;   // the whole (one-problem) workgroup
  }
  if (N > ln) N = 0;
  live = live && N > 0;
  // LDS: per stage vectors of this group's problem
  float* W = lds + (size_t)sub * (fused_lds_floats(ln));   // w = vhat - betahat; restart terms [N][25]
  float* Y = W + ln * V25;        // y = zhat - vhat - e + lamhat [N][25]
  float* ATY = Y + ln * V25;      // Abar^T y                     [N][25]
  float* HT = ATY + ln * V25;     // htilde                       [N][25]
  float* XI = HT + ln * V25;      // xi_{k+1}                     [N][25]
  float* T1 = XI + ln * V25;      // Bt^T w_x + w_u               [N][12]
  float* DU = T1 + ln * NU;       // du                           [N][12]
  float* PIN = DU + ln * NU;      // projection input (u part)    [N][12]
  float* PO = PIN + ln * NU;      // projection output            [N][12]
  float* XI0 = PO + ln * NU;      // [32]

  const int tid = PPW == 1 ? (int)threadIdx.x : (int)threadIdx.x - sub * tpp;
  const bool act = tid < N * NL;
  const int k = act ? tid / NL : 0;
  const int r = act ? tid % NL : 0;
  const size_t s0 = (size_t)b * n;
  const size_t st = s0 + k;
  const float mu = live ? p.mu[b] : 0.f;
  const float tmax = live ? p.tau_max[b] : 0.f;
  const float tsc = live ? ws.tsc[b] : 1.f;

  if (live && tid < NL) {
    float v;
    if (tid < NX) v = p.x0[(size_t)b * NX + tid];
    else v = p.u_prev ? p.u_prev[(size_t)b * NU + tid - NX] /
                            ((tid - NX) % 6 < 3 ? ws.sf[s0] : tsc)
                      : 0.f;
    XI0[tid] = v;
  }

  // operators into registers
  float hrow[NL], o1[NX], o2[NX], o3[NU];
  float qb = 0.f, eb = 0.f;
  if (act) {
    const size_t H0 = st * NH, A0 = st * NX * NX, B0 = st * NX * NU, M0 = st * NM;
    for (int j = 0; j < NL; ++j) hrow[j] = op.h(H0 + pk(r, j, NL));
    if (r < NX) {
      for (int j = 0; j < NX; ++j) o1[j] = op.a(A0 + r * NX + j);    // row r of A
      for (int j = 0; j < NX; ++j) o2[j] = op.a(A0 + j * NX + r);    // column r of A
      for (int j = 0; j < NU; ++j) o3[j] = op.bt(B0 + r * NU + j);   // row r of Bt
    } else {
      const int jj = r - NX;
      for (int i = 0; i < NX; ++i) o1[i] = op.bt(B0 + i * NU + jj);  // column jj of Bt
      for (int i = 0; i < NX; ++i) o2[i] = 0.f;
      for (int l = 0; l < NU; ++l) o3[l] = op.m(M0 + pk(jj, l, NU)); // row jj of M
    }
    qb = ws.qb[st * NL + r];
    eb = (r < NX && p.e) ? p.e[st * NX + r] : 0.f;
  }
  // iterates
  float zh = 0, vh = 0, th = 0, bh = 0, lh = 0;
  float zc = 0, vc = 0, tc = 0, bc = 0, lc = 0;
  if (act) {
    const size_t base = (st * NSTATE) * NL + r;
    zh = ws.hat[base]; vh = ws.hat[base + NL]; th = ws.hat[base + 2 * NL];
    bh = ws.hat[base + 3 * NL]; lh = ws.hat[base + 4 * NL];
    zc = ws.cur[base]; vc = ws.cur[base + NL]; tc = ws.cur[base + 2 * NL];
    bc = ws.cur[base + 3 * NL]; lc = ws.cur[base + 4 * NL];
  }
  float alpha = live ? ws.alpha[b] : 1.f, cprev = live ? ws.cprev[b] : 0.f;
  int restarts = 0;
  const float Fz = live ? p.fz_max[b] : 0.f;
  __syncthreads();

  for (int it = 0; it < iters; ++it) {
    if (act) {
      W[k * V25 + r] = vh - bh;
      Y[k * V25 + r] = zh - vh - eb + lh;
    }
    __syncthreads();
    if (act) {
      const float* y = Y + k * V25;
      float aty;
      if (r < NX) {
        aty = 0.f;
        for (int i = 0; i < NX; ++i) aty = fmaf(o2[i], y[i], aty);
      } else {
        const int jj = r - NX;
        const float* w = W + k * V25;
        aty = y[r];
        float t = w[r];
        for (int i = 0; i < NX; ++i) {
          aty = fmaf(o1[i], y[i], aty);
          t = fmaf(o1[i], w[i], t);
        }
        T1[k * NU + jj] = t;
      }
      ATY[k * V25 + r] = aty;
    }
    __syncthreads();
    if (act) {
      float h = zh - th;
      if (k + 1 < N) h += ATY[(k + 1) * V25 + r];
      HT[k * V25 + r] = fmaf(rho, h, qb);
      if (r >= NX) {
        const float* t = T1 + k * NU;
        float du = 0.f;
        for (int l = 0; l < NU; ++l) du = fmaf(o3[l], t[l], du);
        DU[k * NU + r - NX] = du;
      }
    }
    __syncthreads();
    float xi = 0.f;
    if (act) {
      const float* h = HT + k * V25;
      for (int l = 0; l < NL; ++l) xi = fmaf(hrow[l], h[l], xi);
      XI[k * V25 + r] = xi;
    }
    __syncthreads();
    float s = 0.f, bb = 0.f, gam = 0.f, zin = 0.f;
    if (act) {
      const float* prev = (k == 0) ? XI0 : XI + (k - 1) * V25;
      const float* du = DU + k * NU;
      if (r < NX) {
        for (int j = 0; j < NX; ++j) s = fmaf(o1[j], prev[j], s);
        for (int j = 0; j < NU; ++j) {
          s = fmaf(o3[j], prev[NX + j], s);
          bb = fmaf(o3[j], du[j], bb);
        }
      } else {
        s = prev[r];
        bb = du[r - NX];
      }
      gam = bb + bh - s - eb + lh;
      const float gt = xi + th + s + eb - lh;
      zin = (2.f * gt + gam) * (1.f / 3.f);
      if (r >= NX) PIN[k * NU + r - NX] = zin;
    }
    __syncthreads();
    if (tid < 2 * N) {
      const int kk = tid >> 1, i = tid & 1;
      const float* yv = PIN + kk * NU + 6 * i;
      float* o = PO + kk * NU + 6 * i;
      if (p.contact[(s0 + kk) * 2 + i]) {
        const float F = Fz / ws.sf[s0 + kk];
        const float tm = tmax / tsc;
        float px, py, pz;
        project_pyramid<float>(mu, F, yv[0], yv[1], yv[2], &px, &py, &pz);
        o[0] = px; o[1] = py; o[2] = pz;
        for (int a = 3; a < 6; ++a) o[a] = fminf(fmaxf(yv[a], -tm), tm);
      } else {
        for (int a = 0; a < 6; ++a) o[a] = 0.f;
      }
    }
    __syncthreads();
    float zv = 0, vv = 0, tv = 0, bv = 0, lv = 0;
    if (act) {
      zv = (r < NX) ? zin : PO[k * NU + r - NX];
      vv = 0.5f * (zv + gam);
      tv = th + xi - zv;
      bv = bh + bb - vv;
      lv = lh + zv - s - vv - eb;
      if (accel) {
        const float dz = zv - zh, dv = vv - vh;
        const float d1 = tv - th, d2 = bv - bh, d3 = lv - lh;
        W[k * V25 + r] = d1 * d1 + d2 * d2 + d3 * d3 + dz * dz + dv * dv + (dz - dv) * (dz - dv);
      }
    }
    if (accel) {
      const float cm = stage_ordered_sum(W, T1, N, tid);
      if (cm < eta * cprev) {
        const float an = 0.5f * (1.f + sqrtf(1.f + 4.f * alpha * alpha));
        const float f = (alpha - 1.f) / an;
        zh = zv + f * (zv - zc); vh = vv + f * (vv - vc); th = tv + f * (tv - tc);
        bh = bv + f * (bv - bc); lh = lv + f * (lv - lc);
        alpha = an;
        cprev = cm;
      } else {
        zh = zc; vh = vc; th = tc; bh = bc; lh = lc;
        alpha = 1.f;
        cprev = cprev / eta;
        ++restarts;
      }
      zc = zv; vc = vv; tc = tv; bc = bv; lc = lv;
    } else {
      zh = zv; vh = vv; th = tv; bh = bv; lh = lv;
      __syncthreads();
    }
  }
  if (act) {
    const size_t base = (st * NSTATE) * NL + r;
    ws.hat[base] = zh; ws.hat[base + NL] = vh; ws.hat[base + 2 * NL] = th;
    ws.hat[base + 3 * NL] = bh; ws.hat[base + 4 * NL] = lh;
    if (accel) {
      ws.cur[base] = zc; ws.cur[base + NL] = vc; ws.cur[base + 2 * NL] = tc;
      ws.cur[base + 3 * NL] = bc; ws.cur[base + 4 * NL] = lc;
    }
  }
  if (live && tid == 0) {
    ws.alpha[b] = alpha;
    ws.cprev[b] = cprev;
    ws.restarts[b] += restarts;
  }
}

}  // namespace

// LDS of one problem for a capacity of n stages: five 25-vectors and four
// 12-vectors per stage, then the fixed initial lifted state (32 floats).
size_t fused_lds_bytes(int n) { return fused_lds_floats(n) * sizeof(float); }

// Problems per workgroup that fit: ppw groups of round_up(25 n, 64) threads.
static int fit_ppw(int ppw, int n) {
  const int tpp = ((NL * n + 63) / 64) * 64;
  while (ppw > 1 && ppw * tpp > 1024) ppw /= 2;
  return ppw < 1 ? 1 : ppw;
}

// The instantiation for (threads, precision, problems per workgroup).
#define PINMPC_FUSED_DISPATCH                                           \
  if (threads <= 512) {                                                 \
    if (!s.precision) {                                                 \
      if (ppw == 1) PINMPC_FUSED(512, false, 1);                        \
      else if (ppw == 2) PINMPC_FUSED(512, false, 2);                   \
      else PINMPC_FUSED(512, false, 4);                                 \
    } else {                                                            \
      if (ppw == 1) PINMPC_FUSED(512, true, 1);                         \
      else if (ppw == 2) PINMPC_FUSED(512, true, 2);                    \
      else PINMPC_FUSED(512, true, 4);                                  \
    }                                                                   \
  } else {                                                              \
    if (!s.precision) {                                                 \
      if (ppw == 1) PINMPC_FUSED(1024, false, 1);                       \
      else if (ppw == 2) PINMPC_FUSED(1024, false, 2);                  \
      else PINMPC_FUSED(1024, false, 4);                                \
    } else {                                                            \
      if (ppw == 1) PINMPC_FUSED(1024, true, 1);                        \
      else if (ppw == 2) PINMPC_FUSED(1024, true, 2);                   \
      else PINMPC_FUSED(1024, true, 4);                                 \
    }                                                                   \
  }

hipError_t launch_admm_fused(const Problem& p, const Workspace& w, const pinmpc_settings& s,
                             int iters, hipStream_t st) {
  if (p.batch == 0 || iters == 0) return hipSuccess;
  const int work = NL * p.n_max;
  if (work > 1024) return hipErrorInvalidValue;
  const int ppw = fit_ppw(s.group, p.n_max);
  const int tpp = ((work + 63) / 64) * 64;
  const int threads = ppw * tpp;
  const unsigned grid = (unsigned)((p.batch + ppw - 1) / ppw);
  const size_t lds = (size_t)ppw * fused_lds_bytes(p.n_max);
  // up to 512 threads the kernel may use 256 VGPRs (two waves per SIMD)
#define PINMPC_FUSED(T, BF, G)                                                              \
  hipLaunchKernelGGL((admm_fused_kernel<T, BF, G>), dim3(grid), dim3(threads), lds, st, p, w, \
                     s.rho, s.accel, s.restart_eta, iters, (const int32_t*)nullptr,          \
                     (const int32_t*)nullptr, p.n_max)
  PINMPC_FUSED_DISPATCH
#undef PINMPC_FUSED
  return hipGetLastError();
}

// Problems of horizon class cls, walked through the order array; the grid
// covers the whole batch and workgroups past the class count exit at once.
hipError_t launch_admm_fused_class(const Problem& p, const Workspace& w, const pinmpc_settings& s,
                                   int iters, int cls, hipStream_t st) {
  if (p.batch == 0 || iters == 0) return hipSuccess;
  const int cap = CLASS_N[cls] < p.n_max ? CLASS_N[cls] : p.n_max;
  const int ppw = fit_ppw(s.group, cap);
  const int threads = ppw * (((NL * cap + 63) / 64) * 64);
  const unsigned grid = (unsigned)((p.batch + ppw - 1) / ppw);
  const size_t lds = (size_t)ppw * fused_lds_bytes(cap);
  const int32_t* ord = w.order + (size_t)cls * p.batch;
  const int32_t* cnt = w.counts + cls;
#define PINMPC_FUSED(T, BF, G)                                                                \
  hipLaunchKernelGGL((admm_fused_kernel<T, BF, G>), dim3(grid), dim3(threads), lds, st, p, w, \
                     s.rho, s.accel, s.restart_eta, iters, ord, cnt, cap)
  PINMPC_FUSED_DISPATCH
#undef PINMPC_FUSED
  return hipGetLastError();
}

}  // namespace pinmpc
