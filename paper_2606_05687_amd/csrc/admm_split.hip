// Horizon split across workgroups: the parallel-in-horizon ADMM of Sec. III
// for horizons too long for one workgroup's LDS (up to PINMPC_NMAX_LONG
// stages) or for few problems with long horizons, where the batch alone does
// not fill the chip.
//
// A workgroup owns SEG = 10 consecutive stages of one problem, thread (stage,
// lifted row) as in the one-launch-per-sweep kernel.  The two exchanges the
// splitting leaves cross segment boundaries: block 1 at stage k needs
// Abar_{k+1}^T y_{k+1}, block 2 at stage k needs xi_k from stage k-1 of the
// same sweep.  So one sweep is a chain of launches, each stage-parallel, whose
// outputs go through the workspace:
//   split_p1: y, w of the stage; Abar_k^T y_k and du_k = M_k (Bt^T w_x + w_u)
//   split_p2: htilde_k (needs Abar_{k+1}^T y_{k+1}), xi_{k+1} = H_k htilde_k
//   split_p3: block 2 (needs xi_k), projection, block 3 into the new iterates,
//             and each stage's restart-test term
//   split_p4: per problem, the restart test on the horizon-ordered sum
//   split_p5: extrapolation (or restart) into the next sweep's iterates.
// Every element is computed with the same operations in the same order as in
// the one-launch-per-sweep kernel, so the iterates are bitwise the same.
#include "pinmpc_internal.h"

#pragma clang fp contract(off)

namespace pinmpc {

namespace {

constexpr int SEG = 10;                 // stages per workgroup
constexpr int SPLIT_THREADS = 256;      // SEG x 25 rows active

struct Item {
  int b, k, r, ls, N;
  size_t s0, st;
  bool act;
};

// Workgroup blockIdx.x = b * nseg + segment, nseg = ceil(n_max / SEG).
__device__ inline int seg_count(const Problem& p) { return (p.n_max + SEG - 1) / SEG; }

__device__ inline Item item_of(const Problem& p) {
  Item it;
  const int nseg = seg_count(p);
  it.b = blockIdx.x / nseg;
  it.ls = threadIdx.x / NL;
  it.r = threadIdx.x % NL;
  it.k = (blockIdx.x % nseg) * SEG + it.ls;
  it.N = horizon(p, it.b);
  it.act = it.ls < SEG && it.k < it.N;
  it.s0 = (size_t)it.b * p.n_max;
  it.st = it.s0 + (it.act ? it.k : 0);
  return it;
}

template <bool BF16>
__device__ inline OpLoad<BF16> ops(const Problem& p, const Workspace& ws) {
  OpLoad<BF16> op;
  if constexpr (BF16) {
    op.A = ws.Abf; op.Bt = ws.Btbf; op.H = ws.Hbf; op.M = ws.Mbf;
  } else {
    op.A = p.A; op.Bt = ws.Bt; op.H = ws.Hp; op.M = ws.Mp;
  }
  return op;
}

template <bool BF16>
__global__ void __launch_bounds__(SPLIT_THREADS) split_p1(Problem p, Workspace ws) {
  const Item it = item_of(p);
  const OpLoad<BF16> op = ops<BF16>(p, ws);
  __shared__ float W[SEG][NL], Y[SEG][NL], T[SEG][NU];
  if (it.act) {
    const float* H = ws.hat + (it.st * NSTATE) * NL + it.r;
    const float zh = H[0], vh = H[NL], bh = H[3 * NL], lh = H[4 * NL];
    const float eb = (it.r < NX && p.e) ? p.e[it.st * NX + it.r] : 0.f;
    W[it.ls][it.r] = vh - bh;
    Y[it.ls][it.r] = zh - vh - eb + lh;
  }
  __syncthreads();
  if (it.act) {
    const int r = it.r;
    const size_t A0 = it.st * NX * NX, B0 = it.st * NX * NU;
    const float* w = W[it.ls];
    const float* y = Y[it.ls];
    float acc = 0.f;
    if (r < NX) {
      for (int i = 0; i < NX; ++i) acc = fmaf(op.a(A0 + i * NX + r), y[i], acc);
    } else {
      const int j = r - NX;
      acc = y[r];
      for (int i = 0; i < NX; ++i) acc = fmaf(op.bt(B0 + i * NU + j), y[i], acc);
    }
    ws.sp_aty[it.st * NL + r] = acc;
    if (r < NU) {
      float t = w[NX + r];
      for (int i = 0; i < NX; ++i) t = fmaf(op.bt(B0 + i * NU + r), w[i], t);
      T[it.ls][r] = t;
    }
  }
  __syncthreads();
  if (it.act && it.r < NU) {
    const size_t M0 = it.st * NM;
    float du = 0.f;
    for (int j = 0; j < NU; ++j) du = fmaf(op.m(M0 + pk(it.r, j, NU)), T[it.ls][j], du);
    ws.sp_du[it.st * NU + it.r] = du;
  }
}

template <bool BF16>
__global__ void __launch_bounds__(SPLIT_THREADS) split_p2(Problem p, Workspace ws, float rho) {
  const Item it = item_of(p);
  const OpLoad<BF16> op = ops<BF16>(p, ws);
  __shared__ float HT[SEG][NL];
  if (it.act) {
    const float* H = ws.hat + (it.st * NSTATE) * NL + it.r;
    float h = H[0] - H[2 * NL];
    if (it.k + 1 < it.N) h += ws.sp_aty[(it.st + 1) * NL + it.r];
    HT[it.ls][it.r] = fmaf(rho, h, ws.qb[it.st * NL + it.r]);
  }
  __syncthreads();
  if (it.act) {
    const size_t H0 = it.st * NH;
    float acc = 0.f;
    for (int j = 0; j < NL; ++j) acc = fmaf(op.h(H0 + pk(it.r, j, NL)), HT[it.ls][j], acc);
    ws.sp_xi[it.st * NL + it.r] = acc;
  }
}

template <bool BF16>
__global__ void __launch_bounds__(SPLIT_THREADS) split_p3(Problem p, Workspace ws, int accel) {
  const Item it = item_of(p);
  const OpLoad<BF16> op = ops<BF16>(p, ws);
  __shared__ float PREV[SEG][NL], DU[SEG][NU], PIN[SEG][NU], PO[SEG][NU], CT[SEG][NL];
  const int b = it.b, r = it.r, ls = it.ls;
  if (it.act) {
    float v;
    if (it.k > 0) {
      v = ws.sp_xi[(it.st - 1) * NL + r];
    } else if (r < NX) {
      v = p.x0[(size_t)b * NX + r];
    } else {
      v = p.u_prev ? p.u_prev[(size_t)b * NU + r - NX] /
                         ((r - NX) % 6 < 3 ? ws.sf[it.s0] : ws.tsc[b])
                   : 0.f;
    }
    PREV[ls][r] = v;
    if (r < NU) DU[ls][r] = ws.sp_du[it.st * NU + r];
  }
  __syncthreads();
  float s = 0.f, bb = 0.f, gam = 0.f, zn = 0.f, xi = 0.f, zh = 0.f, vh = 0.f, th = 0.f,
        bh = 0.f, lh = 0.f, eb = 0.f;
  if (it.act) {
    const float* H = ws.hat + (it.st * NSTATE) * NL + r;
    zh = H[0]; vh = H[NL]; th = H[2 * NL]; bh = H[3 * NL]; lh = H[4 * NL];
    eb = (r < NX && p.e) ? p.e[it.st * NX + r] : 0.f;
    xi = ws.sp_xi[it.st * NL + r];
    const float* prev = PREV[ls];
    const float* du = DU[ls];
    if (r < NX) {
      const size_t A0 = it.st * NX * NX + r * NX;
      const size_t B0 = it.st * NX * NU + r * NU;
      for (int j = 0; j < NX; ++j) s = fmaf(op.a(A0 + j), prev[j], s);
      for (int j = 0; j < NU; ++j) {
        const float bt = op.bt(B0 + j);
        s = fmaf(bt, prev[NX + j], s);
        bb = fmaf(bt, du[j], bb);
      }
    } else {
      s = prev[r];
      bb = du[r - NX];
    }
    gam = bb + bh - s - eb + lh;
    const float gt = xi + th + s + eb - lh;
    zn = (2.f * gt + gam) * (1.f / 3.f);
    if (r >= NX) PIN[ls][r - NX] = zn;
  }
  __syncthreads();
  // projection: one thread per (stage, contact) of the segment
  if (threadIdx.x < 2 * SEG) {
    const int l = threadIdx.x >> 1, i = threadIdx.x & 1;
    const int k = (blockIdx.x % seg_count(p)) * SEG + l;
    if (k < it.N) {
      const size_t st = it.s0 + k;
      const float* y = PIN[l] + 6 * i;
      float* o = PO[l] + 6 * i;
      if (p.contact[st * 2 + i]) {
        const float F = p.fz_max[b] / ws.sf[st];
        const float tm = p.tau_max[b] / ws.tsc[b];
        float px, py, pz;
        project_pyramid<float>(p.mu[b], F, y[0], y[1], y[2], &px, &py, &pz);
        o[0] = px; o[1] = py; o[2] = pz;
        for (int a = 3; a < 6; ++a) o[a] = fminf(fmaxf(y[a], -tm), tm);
      } else {
        for (int a = 0; a < 6; ++a) o[a] = 0.f;
      }
    }
  }
  __syncthreads();
  if (it.act) {
    const float z = (r < NX) ? zn : PO[ls][r - NX];
    const float v = 0.5f * (z + gam);
    const float tv = th + xi - z;
    const float bv = bh + bb - v;
    const float lv = lh + z - s - v - eb;
    float* Nw = ws.sp_new + (it.st * NSTATE) * NL + r;
    Nw[0] = z; Nw[NL] = v; Nw[2 * NL] = tv; Nw[3 * NL] = bv; Nw[4 * NL] = lv;
    if (accel) {
      const float dz = z - zh, dv = v - vh;
      const float d1 = tv - th, d2 = bv - bh, d3 = lv - lh;
      CT[ls][r] = d1 * d1 + d2 * d2 + d3 * d3 + dz * dz + dv * dv + (dz - dv) * (dz - dv);
    }
  }
  if (accel) {
    __syncthreads();
    // the stage's term of the restart test: its rows summed in order
    if (threadIdx.x < SEG) {
      const int k = (blockIdx.x % seg_count(p)) * SEG + threadIdx.x;
      if (k < it.N) {
        float a = 0.f;
        for (int rr = 0; rr < NL; ++rr) a += CT[threadIdx.x][rr];
        ws.sp_ct[it.s0 + k] = a;
      }
    }
  }
}

// Restart test of fast ADMM per problem on the horizon-ordered sum of the
// stage terms; writes the extrapolation factor and the restart flag.
__global__ void split_p4(Problem p, Workspace ws, float eta) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= p.batch) return;
  const int N = horizon(p, b);
  const size_t s0 = (size_t)b * p.n_max;
  float cm = 0.f;
  for (int k = 0; k < N; ++k) cm += ws.sp_ct[s0 + k];
  const float cp = ws.cprev[b], al = ws.alpha[b];
  float f = 0.f, restart = 0.f;
  if (cm < eta * cp) {
    const float an = 0.5f * (1.f + sqrtf(1.f + 4.f * al * al));
    f = (al - 1.f) / an;
    ws.alpha[b] = an;
    ws.cprev[b] = cm;
  } else {
    restart = 1.f;
    ws.alpha[b] = 1.f;
    ws.cprev[b] = cp / eta;
    ws.restarts[b] += 1;
  }
  ws.sp_dec[2 * b] = f;
  ws.sp_dec[2 * b + 1] = restart;
}

// Next sweep's iterates: hat from the new iterates (extrapolated, or the
// previous ones on a restart), cur = new.
__global__ void split_p5(Problem p, Workspace ws, int accel) {
  const size_t per = (size_t)NSTATE * NL;
  const size_t total = (size_t)p.batch * p.n_max * per;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int b = (int)(i / ((size_t)p.n_max * per));
    const int k = (int)((i / per) % p.n_max);
    if (k >= horizon(p, b)) continue;
    const float nw = ws.sp_new[i];
    if (accel) {
      const float c = ws.cur[i];
      const float f = ws.sp_dec[2 * b];
      ws.hat[i] = (ws.sp_dec[2 * b + 1] != 0.f) ? c : nw + f * (nw - c);
      ws.cur[i] = nw;
    } else {
      ws.hat[i] = nw;
    }
  }
}

}  // namespace

hipError_t launch_admm_split(const Problem& p, const Workspace& w, const pinmpc_settings& s,
                             int iters, hipStream_t st) {
  if (p.batch == 0 || iters <= 0) return hipSuccess;
  const dim3 grid((unsigned)((size_t)p.batch * ((p.n_max + SEG - 1) / SEG)));
  const size_t items = (size_t)p.batch * p.n_max * NSTATE * NL;
  size_t g5 = (items + 255) / 256;
  if (g5 > 4096) g5 = 4096;
  for (int it = 0; it < iters; ++it) {
    if (s.precision) {
      hipLaunchKernelGGL(split_p1<true>, grid, dim3(SPLIT_THREADS), 0, st, p, w);
      hipLaunchKernelGGL(split_p2<true>, grid, dim3(SPLIT_THREADS), 0, st, p, w, s.rho);
      hipLaunchKernelGGL(split_p3<true>, grid, dim3(SPLIT_THREADS), 0, st, p, w, s.accel);
    } else {
      hipLaunchKernelGGL(split_p1<false>, grid, dim3(SPLIT_THREADS), 0, st, p, w);
      hipLaunchKernelGGL(split_p2<false>, grid, dim3(SPLIT_THREADS), 0, st, p, w, s.rho);
      hipLaunchKernelGGL(split_p3<false>, grid, dim3(SPLIT_THREADS), 0, st, p, w, s.accel);
    }
    if (s.accel)
      hipLaunchKernelGGL(split_p4, dim3((p.batch + 63) / 64), dim3(64), 0, st, p, w,
                         s.restart_eta);
    hipLaunchKernelGGL(split_p5, dim3((unsigned)g5), dim3(256), 0, st, p, w, s.accel);
  }
  return hipGetLastError();
}

}  // namespace pinmpc
