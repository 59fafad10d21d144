// Plain batched form of the parallel-in-horizon ADMM (Sec. III): one kernel
// launch per sweep, operators and iterates streamed from HBM every sweep.
//
// A workgroup owns one problem; thread t handles (stage k, lifted row r),
// r in 0..24 (0..36 with four contacts), so every stage-local update of the
// three blocks runs in parallel across the horizon.  The only cross-stage
// exchanges are the ones the splitting leaves: block 1 at stage k needs Abar_{k+1}^T y_{k+1}
// from stage k+1, block 2 at stage k needs xi_k from stage k-1 of the same
// sweep; both go through LDS.
//
// Slot k of the iterate arrays holds (z_{k+1}, v_k, theta_k, beta_k,
// lambda_k).  Inputs are in scaled coordinates ut = S_k^{-1} u.
#include "pinmpc_internal.h"

// Every multiply-add below is either an explicit fmaf or a separate multiply
// and add: no compiler contraction, so every instantiation of the sweep
// (plain or fused, any block size) computes bitwise the same iterates.
#pragma clang fp contract(off)

namespace pinmpc {

namespace {

struct Lds {     // each buffer: L floats per stage (L = 13 + inputs)
  float* b0;    // w = vhat - betahat           -> later htilde -> restart terms
  float* b1;    // y = zhat - vhat - ebar + lamhat -> later xi (block-1 output)
  float* b2;    // Bt^T w_x + w_u (inputs)      -> later projection input
  float* b3;    // du (inputs)                  -> later projection output
  float* aty;   // Abar^T y of the stage
  float* xi0;   // fixed lifted initial state (x0, ut_prev)
};

// `sweeps` sweeps in one launch: the iterates and the acceleration state stay
// in registers between sweeps (loaded once, stored once); the operators are
// read from memory every sweep.  sweeps = 1 is the plain form.  NC contacts
// per stage (2: feet, 4: feet and hands).
template <int PAIRS, bool BF16, int NC>
__global__ void __launch_bounds__(1024) admm_sweep_kernel(Problem p, Workspace ws, float rho,
                                                          int accel, float eta,
                                                          const int32_t* order,
                                                          const int32_t* count, int sweeps) {
  constexpr int NU = Dims<NC>::U, NL = Dims<NC>::L, NH = Dims<NC>::H, NM = Dims<NC>::M;
  constexpr int BUF = NL;
  if (count && (int)blockIdx.x >= *count) return;
  OpLoad<BF16> op;
  if constexpr (BF16) {
    op.A = ws.Abf; op.Bt = ws.Btbf; op.H = ws.Hbf; op.M = ws.Mbf;
  } else {
    op.A = p.A; op.Bt = ws.Bt; op.H = ws.Hp; op.M = ws.Mp;
  }
  extern __shared__ float lds[];
  const int b = order ? order[blockIdx.x] : (int)blockIdx.x;
  const int n = p.n_max;
  const int N = horizon(p, b);
  Lds L;
  L.b0 = lds;
  L.b1 = L.b0 + n * BUF;
  L.b2 = L.b1 + n * BUF;
  L.b3 = L.b2 + n * BUF;
  L.aty = L.b3 + n * BUF;
  L.xi0 = L.aty + n * BUF;
  const int nact = N * NL;
  const size_t s0 = (size_t)b * n;
  const float* e = p.e;
  const float mu = p.mu[b];
  const float tmax = p.tau_max[b];

  if (threadIdx.x < NL) {
    const int r = threadIdx.x;
    float v;
    if (r < NX) v = p.x0[(size_t)b * NX + r];
    else v = p.u_prev ? p.u_prev[(size_t)b * NU + r - NX] /
                            ((r - NX) % 6 < 3 ? ws.sf[s0] : ws.tsc[b])
                      : 0.f;
    L.xi0[r] = v;
  }

  float zh[PAIRS], vh[PAIRS], th[PAIRS], bh[PAIRS], lh[PAIRS];
  float zc[PAIRS], vc[PAIRS], tc[PAIRS], bc[PAIRS], lc[PAIRS];
  float xi[PAIRS], sv[PAIRS], bv[PAIRS], gam[PAIRS], zn[PAIRS], eb[PAIRS];

#pragma unroll
  for (int q = 0; q < PAIRS; ++q) {
    const int id = threadIdx.x + q * blockDim.x;
    if (id < nact) {
      const int k = id / NL, r = id % NL;
      const size_t base = ((s0 + k) * NSTATE) * NL + r;
      const float* H = ws.hat + base;
      zh[q] = H[0]; vh[q] = H[NL]; th[q] = H[2 * NL]; bh[q] = H[3 * NL]; lh[q] = H[4 * NL];
      if (accel) {
        const float* C = ws.cur + base;
        zc[q] = C[0]; vc[q] = C[NL]; tc[q] = C[2 * NL]; bc[q] = C[3 * NL]; lc[q] = C[4 * NL];
      }
      eb[q] = (r < NX && e) ? e[(s0 + k) * NX + r] : 0.f;
    }
  }
  float al = ws.alpha[b], cp = ws.cprev[b];
  int nrest = 0;

  for (int it = 0; it < sweeps; ++it) {
#pragma unroll
  for (int q = 0; q < PAIRS; ++q) {
    const int id = threadIdx.x + q * blockDim.x;
    if (id < nact) {
      const int k = id / NL, r = id % NL;
      L.b0[k * BUF + r] = vh[q] - bh[q];
      L.b1[k * BUF + r] = zh[q] - vh[q] - eb[q] + lh[q];
    }
  }
  __syncthreads();

  // Block 1a: Bt^T w_x + w_u and Abar_k^T y_k (stage-local).
#pragma unroll
  for (int q = 0; q < PAIRS; ++q) {
    const int id = threadIdx.x + q * blockDim.x;
    if (id < nact) {
      const int k = id / NL, r = id % NL;
      const size_t A0 = (s0 + k) * NX * NX;
      const size_t B0 = (s0 + k) * NX * NU;
      const float* w = L.b0 + k * BUF;
      const float* y = L.b1 + k * BUF;
      float acc = 0.f;
      if (r < NX) {
        for (int i = 0; i < NX; ++i) acc = fmaf(op.a(A0 + i * NX + r), y[i], acc);
      } else {
        const int j = r - NX;
        acc = y[r];
        for (int i = 0; i < NX; ++i) acc = fmaf(op.bt(B0 + i * NU + j), y[i], acc);
      }
      L.aty[k * BUF + r] = acc;
      if (r < NU) {
        float t = w[NX + r];
        for (int i = 0; i < NX; ++i) t = fmaf(op.bt(B0 + i * NU + r), w[i], t);
        L.b2[k * BUF + r] = t;
      }
    }
  }
  __syncthreads();

  // Block 1b: du_k = M_k t,  htilde_k = qbar + rho (zhat - thetahat + Abar_{k+1}^T y_{k+1}).
  float ht[PAIRS];
#pragma unroll
  for (int q = 0; q < PAIRS; ++q) {
    const int id = threadIdx.x + q * blockDim.x;
    if (id < nact) {
      const int k = id / NL, r = id % NL;
      float h = zh[q] - th[q];
      if (k + 1 < N) h += L.aty[(k + 1) * BUF + r];
      ht[q] = fmaf(rho, h, ws.qb[(s0 + k) * NL + r]);
      if (r < NU) {
        const size_t M0 = (s0 + k) * NM;
        const float* t = L.b2 + k * BUF;
        float du = 0.f;
        for (int j = 0; j < NU; ++j) du = fmaf(op.m(M0 + pk(r, j, NU)), t[j], du);
        L.b3[k * BUF + r] = du;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PAIRS; ++q) {
    const int id = threadIdx.x + q * blockDim.x;
    if (id < nact) {
      const int k = id / NL, r = id % NL;
      L.b0[k * BUF + r] = ht[q];
    }
  }
  __syncthreads();

  // Block 1c: xi_{k+1} = H_k htilde_k.
#pragma unroll
  for (int q = 0; q < PAIRS; ++q) {
    const int id = threadIdx.x + q * blockDim.x;
    if (id < nact) {
      const int k = id / NL, r = id % NL;
      const size_t H0 = (s0 + k) * NH;
      const float* h = L.b0 + k * BUF;
      float acc = 0.f;
      for (int j = 0; j < NL; ++j) acc = fmaf(op.h(H0 + pk(r, j, NL)), h[j], acc);
      xi[q] = acc;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PAIRS; ++q) {
    const int id = threadIdx.x + q * blockDim.x;
    if (id < nact) {
      const int k = id / NL, r = id % NL;
      L.b1[k * BUF + r] = xi[q];
    }
  }
  __syncthreads();

  // Block 2: s_k = Abar_k xi_k (xi_k of this sweep, xi_0 fixed), b_k = Bbar_k du_k,
  // z_{k+1} = Proj((2 gamtilde + gam) / 3), v_k = (z_{k+1} + gam) / 2.
#pragma unroll
  for (int q = 0; q < PAIRS; ++q) {
    const int id = threadIdx.x + q * blockDim.x;
    if (id < nact) {
      const int k = id / NL, r = id % NL;
      const float* prev = (k == 0) ? L.xi0 : L.b1 + (k - 1) * BUF;
      const float* du = L.b3 + k * BUF;
      float s, bb;
      if (r < NX) {
        const size_t A0 = (s0 + k) * NX * NX + r * NX;
        const size_t B0 = (s0 + k) * NX * NU + r * NU;
        s = 0.f;
        for (int j = 0; j < NX; ++j) s = fmaf(op.a(A0 + j), prev[j], s);
        bb = 0.f;
        for (int j = 0; j < NU; ++j) {
          const float bt = op.bt(B0 + j);
          s = fmaf(bt, prev[NX + j], s);
          bb = fmaf(bt, du[j], bb);
        }
      } else {
        s = prev[r];
        bb = du[r - NX];
      }
      sv[q] = s;
      bv[q] = bb;
      gam[q] = bb + bh[q] - s - eb[q] + lh[q];
      const float gt = xi[q] + th[q] + s + eb[q] - lh[q];
      zn[q] = (2.f * gt + gam[q]) * (1.f / 3.f);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PAIRS; ++q) {
    const int id = threadIdx.x + q * blockDim.x;
    if (id < nact) {
      const int k = id / NL, r = id % NL;
      if (r >= NX) L.b2[k * BUF + r - NX] = zn[q];
    }
  }
  __syncthreads();
  // projection: one thread per (stage, contact)
  for (int id = threadIdx.x; id < N * NC; id += blockDim.x) {
    const int k = id / NC, i = id % NC;
    const float* y = L.b2 + k * BUF + 6 * i;
    float* o = L.b3 + k * BUF + 6 * i;
    if (p.contact[(s0 + k) * NC + i]) {
      const float sf = ws.sf[s0 + k];
      const float F = p.fz_max[b] / sf;
      const float tm = tmax / ws.tsc[b];
      float px, py, pz;
      project_pyramid<float>(mu, F, y[0], y[1], y[2], &px, &py, &pz);
      o[0] = px; o[1] = py; o[2] = pz;
      for (int a = 3; a < 6; ++a) o[a] = fminf(fmaxf(y[a], -tm), tm);
    } else {
      for (int a = 0; a < 6; ++a) o[a] = 0.f;
    }
  }
  __syncthreads();

  // Block 3 and the acceleration test.
  float zv[PAIRS], vv[PAIRS], tv[PAIRS], bvv[PAIRS], lv[PAIRS];
#pragma unroll
  for (int q = 0; q < PAIRS; ++q) {
    const int id = threadIdx.x + q * blockDim.x;
    if (id < nact) {
      const int k = id / NL, r = id % NL;
      const float z = (r < NX) ? zn[q] : L.b3[k * BUF + r - NX];
      const float v = 0.5f * (z + gam[q]);
      zv[q] = z;
      vv[q] = v;
      tv[q] = th[q] + xi[q] - z;
      bvv[q] = bh[q] + bv[q] - v;
      lv[q] = lh[q] + z - sv[q] - v - eb[q];
      if (accel) {
        const float dz = z - zh[q], dv = v - vh[q];
        const float d1 = tv[q] - th[q], d2 = bvv[q] - bh[q], d3 = lv[q] - lh[q];
        L.b0[k * BUF + r] =
            d1 * d1 + d2 * d2 + d3 * d3 + dz * dz + dv * dv + (dz - dv) * (dz - dv);
      }
    }
  }
  float f = 0.f;
  bool restart = false;
  if (accel) {
    const float cm = stage_ordered_sum<NL>(L.b0, L.b2, N, threadIdx.x);
    if (cm < eta * cp) {
      const float an = 0.5f * (1.f + sqrtf(1.f + 4.f * al * al));
      f = (al - 1.f) / an;
      al = an;
      cp = cm;
    } else {
      restart = true;
      al = 1.f;
      cp = cp / eta;
      ++nrest;
    }
  }
#pragma unroll
  for (int q = 0; q < PAIRS; ++q) {
    if (accel) {
      if (restart) {
        zh[q] = zc[q]; vh[q] = vc[q]; th[q] = tc[q]; bh[q] = bc[q]; lh[q] = lc[q];
      } else {
        zh[q] = zv[q] + f * (zv[q] - zc[q]);
        vh[q] = vv[q] + f * (vv[q] - vc[q]);
        th[q] = tv[q] + f * (tv[q] - tc[q]);
        bh[q] = bvv[q] + f * (bvv[q] - bc[q]);
        lh[q] = lv[q] + f * (lv[q] - lc[q]);
      }
      zc[q] = zv[q]; vc[q] = vv[q]; tc[q] = tv[q]; bc[q] = bvv[q]; lc[q] = lv[q];
    } else {
      zh[q] = zv[q]; vh[q] = vv[q]; th[q] = tv[q]; bh[q] = bvv[q]; lh[q] = lv[q];
    }
  }
  __syncthreads();   // this sweep's LDS reads are done before the next one writes
  }  // sweeps

#pragma unroll
  for (int q = 0; q < PAIRS; ++q) {
    const int id = threadIdx.x + q * blockDim.x;
    if (id < nact) {
      const int k = id / NL, r = id % NL;
      const size_t base = ((s0 + k) * NSTATE) * NL + r;
      float* H = ws.hat + base;
      H[0] = zh[q]; H[NL] = vh[q]; H[2 * NL] = th[q]; H[3 * NL] = bh[q]; H[4 * NL] = lh[q];
      if (accel) {
        float* C = ws.cur + base;
        C[0] = zc[q]; C[NL] = vc[q]; C[2 * NL] = tc[q]; C[3 * NL] = bc[q]; C[4 * NL] = lc[q];
      }
    }
  }
  if (threadIdx.x == 0 && accel) {
    ws.alpha[b] = al;
    ws.cprev[b] = cp;
    ws.restarts[b] += nrest;
  }
}

// Initial iterates: zero, or (warm start) the stored iterates of the
// problem's slot shifted by one stage (slot k takes stored slot k+1, the last
// stage repeats).  Acceleration state restarts.
__global__ void admm_init_kernel(Problem p, Workspace ws) {
  const int NL = NX + 6 * p.nc;
  const size_t total = (size_t)p.batch * p.n_max * NSTATE * NL;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    float v = 0.f;
    if (ws.warm_idx) {
      const size_t per = (size_t)NSTATE * NL;
      const int b = (int)(i / ((size_t)p.n_max * per));
      const int k = (int)((i / per) % p.n_max);
      const int e = (int)(i % per);
      const int slot = ws.warm_idx[b];
      const int N = horizon(p, b);
      if (slot >= 0 && k < N) {
        const int ks = (k + 1 < N) ? k + 1 : N - 1;
        v = ws.warm_store[((size_t)slot * PINMPC_NMAX + ks) * per + e];
      }
    }
    ws.cur[i] = v;
    ws.hat[i] = v;
  }
  for (size_t b = (size_t)blockIdx.x * blockDim.x + threadIdx.x; b < (size_t)p.batch;
       b += (size_t)gridDim.x * blockDim.x) {
    ws.alpha[b] = 1.f;
    ws.cprev[b] = 3.0e38f;
    ws.restarts[b] = 0;
  }
}

// Store the final iterates of warm-started problems into their slots.
__global__ void warm_save_kernel(Problem p, Workspace ws, int accel) {
  const int NL = NX + 6 * p.nc;
  const size_t per = (size_t)NSTATE * NL;
  const size_t total = (size_t)p.batch * p.n_max * per;
  const float* src = accel ? ws.cur : ws.hat;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int b = (int)(i / ((size_t)p.n_max * per));
    const int k = (int)((i / per) % p.n_max);
    const int slot = ws.warm_idx[b];
    if (slot < 0 || k >= horizon(p, b)) continue;
    ws.warm_store[((size_t)slot * PINMPC_NMAX + k) * per + i % per] = src[i];
  }
}

__global__ void fill_i32_kernel(int32_t* dst, size_t n, int32_t base, int32_t step) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = base + step * (int32_t)i;
}

// z iterates (current) in unscaled coordinates, [b][n_max][13 + inputs].
__global__ void admm_extract_kernel(Problem p, Workspace ws, int accel, float* z_out) {
  const int NL = NX + 6 * p.nc;
  const size_t total = (size_t)p.batch * p.n_max * NL;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const size_t s = i / NL;
    const int r = (int)(i % NL);
    const int b = (int)(s / p.n_max);
    const float* src = accel ? ws.cur : ws.hat;
    float v = src[s * NSTATE * NL + r];
    if (r >= NX) v *= ((r - NX) % 6 < 3) ? ws.sf[s] : ws.tsc[b];
    z_out[i] = v;
  }
}

}  // namespace

hipError_t launch_admm_init(const Problem& p, const Workspace& w, hipStream_t st) {
  if (p.batch == 0) return hipSuccess;
  hipLaunchKernelGGL(admm_init_kernel, dim3(1024), dim3(256), 0, st, p, w);
  return hipGetLastError();
}

hipError_t launch_warm_save(const Problem& p, const Workspace& w, int accel, hipStream_t st) {
  if (p.batch == 0 || !w.warm_idx) return hipSuccess;
  hipLaunchKernelGGL(warm_save_kernel, dim3(1024), dim3(256), 0, st, p, w, accel);
  return hipGetLastError();
}

static unsigned grid_for(size_t n) {
  size_t g = (n + 255) / 256;
  if (g > 2048) g = 2048;
  return (unsigned)(g ? g : 1);
}

hipError_t launch_fill_i32(int32_t* dst, size_t n, int32_t base, int32_t step, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(n)), dim3(256), 0, st, dst, n, base, step);
  return hipGetLastError();
}

static hipError_t sweep(const Problem& p, const Workspace& w, const pinmpc_settings& s,
                        const int32_t* ord, const int32_t* cnt, int sweeps, hipStream_t st) {
  if (p.batch == 0) return hipSuccess;
  const int nl = NX + 6 * p.nc;
  const int work = nl * p.n_max;
  int threads = ((work + 63) / 64) * 64;
  if (threads > 1024) threads = 1024;
  const int pairs = (work + threads - 1) / threads;
  // five stage buffers and the initial lifted state
  const size_t lds = (size_t)(5 * p.n_max * nl + 64) * sizeof(float);
#define PINMPC_SWEEP(P, BF, C)                                                              \
  hipLaunchKernelGGL((admm_sweep_kernel<P, BF, C>), dim3(p.batch), dim3(threads), lds, st, p, \
                     w, s.rho, s.accel, s.restart_eta, ord, cnt, sweeps)
  const bool bf = s.precision != 0;
  if (p.nc == 2) {
    if (pairs == 1 && !bf) PINMPC_SWEEP(1, false, 2);
    else if (pairs == 1) PINMPC_SWEEP(1, true, 2);
    else if (pairs == 2 && !bf) PINMPC_SWEEP(2, false, 2);
    else if (pairs == 2) PINMPC_SWEEP(2, true, 2);
    else return hipErrorInvalidValue;
  } else if (p.nc == 4) {
    if (pairs == 1 && !bf) PINMPC_SWEEP(1, false, 4);
    else if (pairs == 1) PINMPC_SWEEP(1, true, 4);
    else if (pairs == 2 && !bf) PINMPC_SWEEP(2, false, 4);
    else if (pairs == 2) PINMPC_SWEEP(2, true, 4);
    else if (pairs == 3 && !bf) PINMPC_SWEEP(3, false, 4);
    else if (pairs == 3) PINMPC_SWEEP(3, true, 4);
    else return hipErrorInvalidValue;
  } else {
    return hipErrorInvalidValue;
  }
#undef PINMPC_SWEEP
  return hipGetLastError();
}

hipError_t launch_admm_sweep(const Problem& p, const Workspace& w, const pinmpc_settings& s,
                             int sweeps, hipStream_t st) {
  return sweep(p, w, s, nullptr, nullptr, sweeps, st);
}

hipError_t launch_admm_sweep_class(const Problem& p, const Workspace& w,
                                   const pinmpc_settings& s, int cls, int sweeps,
                                   hipStream_t st) {
  return sweep(p, w, s, w.order + (size_t)cls * p.batch, w.counts + cls, sweeps, st);
}

namespace {

__global__ void zero_counts_kernel(int32_t* counts) {
  if (threadIdx.x < 4) counts[threadIdx.x] = 0;
}

__global__ void classify_kernel(Problem p, Workspace ws) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= p.batch) return;
  const int N = horizon(p, b);
  const int cls = N <= CLASS_N[0] ? 0 : (N <= CLASS_N[1] ? 1 : 2);
  const int slot = atomicAdd(ws.counts + cls, 1);
  ws.order[(size_t)cls * p.batch + slot] = b;
}

}  // namespace

hipError_t launch_classify(const Problem& p, const Workspace& w, hipStream_t st) {
  if (p.batch == 0) return hipSuccess;
  hipLaunchKernelGGL(zero_counts_kernel, dim3(1), dim3(64), 0, st, w.counts);
  hipLaunchKernelGGL(classify_kernel, dim3((p.batch + 255) / 256), dim3(256), 0, st, p, w);
  return hipGetLastError();
}

hipError_t launch_admm_extract(const Problem& p, const Workspace& w, int accel,
                               float* z_out, hipStream_t st) {
  if (p.batch == 0) return hipSuccess;
  hipLaunchKernelGGL(admm_extract_kernel, dim3(1024), dim3(256), 0, st, p, w, accel, z_out);
  return hipGetLastError();
}

}  // namespace pinmpc
