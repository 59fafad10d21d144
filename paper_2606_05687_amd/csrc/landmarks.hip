// The step after the solve: MPC landmark guidance reward (Sec. II-C).
//
// Every solve at tick T stores, per environment, the predicted CoM at the
// landmark offsets n_l = 1 + floor(s_l (N - 1)), s_l = l / (N_L - 1), i.e. at
// ticks T + n_l d (d ticks per MPC step); when the rollout reaches tick t, the
// realised CoM is compared with every landmark predicted for t, and
//   r_t = exp(-sum_l alpha_l |c_t - c_hat_l|_Qc^2 / sigma^2),
// landmarks that were never predicted for t being left out.
//
// Store: per environment a ring of R slots indexed by target tick mod R, each
// slot holding N_L landmarks (CoM, 3 floats) and the target tick each was
// stored for (int32; -1 = empty).  A slot is read at tick t only if its tag
// equals t, so stale entries from earlier ticks or episodes are never used.
// R > N_max d keeps a landmark until its tick arrives.  Environments are
// independent and the kernels are tiny (tens of bytes per environment): one
// thread per (environment, landmark) or per environment.
#include "pinmpc_internal.h"

namespace pinmpc {

namespace {

__device__ inline int landmark_offset(int l, int n_l, int N) {
  if (n_l == 1) return 1;
  // 1 + floor(l (N - 1) / (N_L - 1)) in exact integer arithmetic
  return 1 + (l * (N - 1)) / (n_l - 1);
}

__global__ void landmarks_clear_kernel(LandmarkStore st, const uint8_t* mask) {
  const size_t per = (size_t)st.ring * st.n_landmarks;
  const size_t total = (size_t)st.envs * per;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    if (mask && !mask[i / per]) continue;
    st.tag[i] = -1;
  }
}

__global__ void landmarks_push_kernel(LandmarkStore st, int n_max, const int32_t* N,
                                      const float* x, int32_t tick) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= st.envs * st.n_landmarks) return;
  const int e = i / st.n_landmarks, l = i % st.n_landmarks;
  int Ne = N ? N[e] : n_max;
  if (Ne < 1 || Ne > n_max) return;           // no trajectory to take landmarks from
  const int n = landmark_offset(l, st.n_landmarks, Ne);
  const int target = tick + n * st.ticks_per_step;
  const int slot = target % st.ring;
  const size_t at = ((size_t)e * st.ring + slot) * st.n_landmarks + l;
  const float* xs = x + ((size_t)e * (n_max + 1) + n) * NX;
  st.com[3 * at + 0] = xs[3];
  st.com[3 * at + 1] = xs[4];
  st.com[3 * at + 2] = xs[5];
  st.tag[at] = target;
}

__global__ void landmark_reward_kernel(LandmarkStore st, const float* com, int32_t tick,
                                       const float* alpha, const float* qc, float inv_s2,
                                       float* reward, int32_t* used) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= st.envs) return;
  const int slot = tick % st.ring;
  const float cx = com[3 * e], cy = com[3 * e + 1], cz = com[3 * e + 2];
  float acc = 0.f;
  int bits = 0;
  for (int l = 0; l < st.n_landmarks; ++l) {
    const size_t at = ((size_t)e * st.ring + slot) * st.n_landmarks + l;
    if (st.tag[at] != tick) continue;
    const float ex = cx - st.com[3 * at], ey = cy - st.com[3 * at + 1],
                ez = cz - st.com[3 * at + 2];
    acc += alpha[l] * (qc[0] * ex * ex + qc[1] * ey * ey + qc[2] * ez * ez);
    bits |= 1 << l;
  }
  reward[e] = expf(-acc * inv_s2);
  if (used) used[e] = bits;
}

unsigned grid1(size_t n) {
  size_t g = (n + 255) / 256;
  return (unsigned)(g ? (g > 65535 ? 65535 : g) : 1);
}

}  // namespace

hipError_t launch_landmarks_clear(const LandmarkStore& st, const uint8_t* mask, hipStream_t s) {
  if (st.envs == 0) return hipSuccess;
  hipLaunchKernelGGL(landmarks_clear_kernel, dim3(grid1((size_t)st.envs * st.ring * st.n_landmarks)),
                     dim3(256), 0, s, st, mask);
  return hipGetLastError();
}

hipError_t launch_landmarks_push(const LandmarkStore& st, int n_max, const int32_t* N,
                                 const float* x, int32_t tick, hipStream_t s) {
  if (st.envs == 0) return hipSuccess;
  const size_t n = (size_t)st.envs * st.n_landmarks;
  hipLaunchKernelGGL(landmarks_push_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     st, n_max, N, x, tick);
  return hipGetLastError();
}

hipError_t launch_landmark_reward(const LandmarkStore& st, const float* com, int32_t tick,
                                  const float* alpha, const float* qc, float sigma,
                                  float* reward, int32_t* used, hipStream_t s) {
  if (st.envs == 0) return hipSuccess;
  hipLaunchKernelGGL(landmark_reward_kernel, dim3((unsigned)((st.envs + 255) / 256)), dim3(256),
                     0, s, st, com, tick, alpha, qc, 1.f / (sigma * sigma), reward, used);
  return hipGetLastError();
}

}  // namespace pinmpc
