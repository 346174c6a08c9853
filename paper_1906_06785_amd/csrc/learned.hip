// Learned correction of the mean spatial solve: device kernels and training.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <random>
#include <stdexcept>
#include <string>
#include <vector>

#include "learned.h"

namespace sgtt {

namespace {

#define MLP_HIP(x)                                                                                  \
  do {                                                                                              \
    hipError_t e_ = (x);                                                                            \
    if (e_ != hipSuccess) throw std::runtime_error(std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

inline unsigned cdivu(long a, long b) { return (unsigned)((a + b - 1) / b); }

typedef float f4v __attribute__((ext_vector_type(4)));

template <class T>
__device__ __forceinline__ float ldf(const T* p, long i) {
  return (float)p[i];
}
template <>
__device__ __forceinline__ float ldf<unsigned short>(const unsigned short* p, long i) {
  return __half2float(__ushort_as_half(p[i]));
}

constexpr int MT = 64, MK = 16;

// C(i,j) = alpha * sum_k A(i,k) B(k,j) + beta * C(i,j) with general strides,
// A of type TA (FP16 bits, float or double), B of type TB; operands rounded
// to FP32 and multiplied on the matrix cores (v_mfma_f32_16x16x4f32: lane l
// supplies A[l%16][l/16] and B[l/16][l%16]; accumulator item v is
// D[4(l/16) + v][l%16]) with FP32 accumulation.  64 x 64 tile per
// 256-thread workgroup, each wave a 32 x 32 quarter.
template <class TA, class TB, class TC>
__global__ __launch_bounds__(256) void k_mgemm(int m, int n, int k, float alpha, const TA* __restrict__ A, long sAi,
                                               long sAk, const TB* __restrict__ B, long sBk, long sBj, float beta,
                                               TC* __restrict__ C, long sCi, long sCj) {
  __shared__ float As[MK][MT + 1];
  __shared__ float Bs[MK][MT + 1];
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int i0 = blockIdx.y * MT, j0 = blockIdx.x * MT;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int lr = lane % 16, lk = lane / 16;
  f4v acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f4v{0.f, 0.f, 0.f, 0.f};
  const bool a_kfast = (sAk == 1), b_kfast = (sBk == 1);
  for (int kk = 0; kk < k; kk += MK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      int ii, kx;
      if (a_kfast) { kx = e % MK; ii = e / MK; } else { ii = e % MT; kx = e / MT; }
      const long gi = i0 + ii, gk = kk + kx;
      As[kx][ii] = (gi < m && gk < k) ? ldf(A, gi * sAi + gk * sAk) : 0.f;
      int jj, kx2;
      if (b_kfast) { kx2 = e % MK; jj = e / MK; } else { jj = e % MT; kx2 = e / MT; }
      const long gj = j0 + jj, gk2 = kk + kx2;
      Bs[kx2][jj] = (gj < n && gk2 < k) ? ldf(B, gk2 * sBk + gj * sBj) : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kq = 0; kq < MK / 4; ++kq) {
      const int kr = kq * 4 + lk;
      const float a0 = As[kr][wr + lr], a1 = As[kr][wr + 16 + lr];
      const float b0 = Bs[kr][wc + lr], b1 = Bs[kr][wc + 16 + lr];
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int tr = 0; tr < 2; ++tr)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const long gi = i0 + wr + tr * 16 + 4 * lk + v;
      if (gi >= m) continue;
#pragma unroll
      for (int tc = 0; tc < 2; ++tc) {
        const long gj = j0 + wc + tc * 16 + lr;
        if (gj >= n) continue;
        TC* cp = C + gi * sCi + gj * sCj;
        float val = alpha * acc[tr][tc][v];
        if (beta != 0.f) val += beta * (float)(*cp);
        *cp = (TC)val;
      }
    }
}

// The same product with FP16 operands on the FP16 matrix cores
// (v_mfma_f32_16x16x16f16, FP32 accumulation): A (FP16 weight bits) is exact
// in FP16; B is scaled by bscale[j] (when given) and rounded to FP16 as it is
// staged.  Lane l supplies A[l%16][4(l/16) .. 4(l/16)+3] and
// B[4(l/16) .. 4(l/16)+3][l%16]; accumulator item v is D[4(l/16) + v][l%16].
// The tiles sit in LDS with k contiguous (rows of MK + 4 halves), so a lane
// reads its four operands as one 8-byte load.
typedef _Float16 h4v __attribute__((ext_vector_type(4)));

template <class TA, class TB, class TC>
__global__ __launch_bounds__(256) void k_mgemm_h(int m, int n, int k, float alpha, const TA* __restrict__ A, long sAi,
                                                 long sAk, const TB* __restrict__ B, long sBk, long sBj,
                                                 const float* __restrict__ bscale, float beta, TC* __restrict__ C,
                                                 long sCi, long sCj) {
  constexpr int KP = MK + 4;
  __shared__ __align__(16) _Float16 Ah[MT * KP];
  __shared__ __align__(16) _Float16 Bh[MT * KP];
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int i0 = blockIdx.y * MT, j0 = blockIdx.x * MT;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int lr = lane % 16, lk = lane / 16;
  f4v acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f4v{0.f, 0.f, 0.f, 0.f};
  const bool a_kfast = (sAk == 1), b_kfast = (sBk == 1);
  for (int kk = 0; kk < k; kk += MK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      int ii, kx;
      if (a_kfast) { kx = e % MK; ii = e / MK; } else { ii = e % MT; kx = e / MT; }
      const long gi = i0 + ii, gk = kk + kx;
      Ah[ii * KP + kx] = (_Float16)((gi < m && gk < k) ? ldf(A, gi * sAi + gk * sAk) : 0.f);
      int jj, kx2;
      if (b_kfast) { kx2 = e % MK; jj = e / MK; } else { jj = e % MT; kx2 = e / MT; }
      const long gj = j0 + jj, gk2 = kk + kx2;
      float bv = (gj < n && gk2 < k) ? ldf(B, gk2 * sBk + gj * sBj) : 0.f;
      if (bscale && gj < n) bv *= bscale[gj];
      Bh[jj * KP + kx2] = (_Float16)bv;
    }
    __syncthreads();
    const h4v a0 = *reinterpret_cast<const h4v*>(&Ah[(wr + lr) * KP + 4 * lk]);
    const h4v a1 = *reinterpret_cast<const h4v*>(&Ah[(wr + 16 + lr) * KP + 4 * lk]);
    const h4v b0 = *reinterpret_cast<const h4v*>(&Bh[(wc + lr) * KP + 4 * lk]);
    const h4v b1 = *reinterpret_cast<const h4v*>(&Bh[(wc + 16 + lr) * KP + 4 * lk]);
    acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x16f16(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x16f16(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x16f16(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x16f16(a1, b1, acc[1][1], 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int tr = 0; tr < 2; ++tr)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const long gi = i0 + wr + tr * 16 + 4 * lk + v;
      if (gi >= m) continue;
#pragma unroll
      for (int tc = 0; tc < 2; ++tc) {
        const long gj = j0 + wc + tc * 16 + lr;
        if (gj >= n) continue;
        TC* cp = C + gi * sCi + gj * sCj;
        float val = alpha * acc[tr][tc][v];
        if (beta != 0.f) val += beta * (float)(*cp);
        *cp = (TC)val;
      }
    }
}

template <class TA, class TB, class TC>
void mgemm_h(hipStream_t s, int m, int n, int k, float alpha, const TA* A, long sAi, long sAk, const TB* B, long sBk,
             long sBj, const float* bscale, float beta, TC* C, long sCi, long sCj) {
  if (m <= 0 || n <= 0) return;
  hipLaunchKernelGGL((k_mgemm_h<TA, TB, TC>), dim3(cdivu(n, MT), cdivu(m, MT)), dim3(256), 0, s, m, n, k, alpha, A,
                     sAi, sAk, B, sBk, sBj, bscale, beta, C, sCi, sCj);
}

template <class TA, class TB, class TC>
void mgemm(hipStream_t s, int m, int n, int k, float alpha, const TA* A, long sAi, long sAk, const TB* B, long sBk,
           long sBj, float beta, TC* C, long sCi, long sCj) {
  if (m <= 0 || n <= 0) return;
  hipLaunchKernelGGL((k_mgemm<TA, TB, TC>), dim3(cdivu(n, MT), cdivu(m, MT)), dim3(256), 0, s, m, n, k, alpha, A, sAi,
                     sAk, B, sBk, sBj, beta, C, sCi, sCj);
}

__device__ double block_sum_d(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    for (int q = 0; q < (int)(blockDim.x / 64); ++q) t += sh[q];
    sh[0] = t;
  }
  __syncthreads();
  t = sh[0];
  __syncthreads();
  return t;
}

// Z (rows x cols, column j at Z + j*rows) = act(Z * colscale[j] + b[i])
__global__ void k_bias_act(int rows, int cols, float* __restrict__ Z, const float* __restrict__ b,
                           const float* __restrict__ colscale, int relu) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)rows * cols) return;
  const int i = e % rows, j = e / rows;
  float v = Z[e];
  if (colscale) v *= colscale[j];
  v += b[i];
  Z[e] = (relu && v < 0.f) ? 0.f : v;
}

// dZ *= (H > 0)
__global__ void k_relu_bwd(long n, float* __restrict__ dZ, const float* __restrict__ H) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n && !(H[e] > 0.f)) dZ[e] = 0.f;
}

// out[i] = sum_j M[j*rows + i]
__global__ void k_rowsum(int rows, int cols, const float* __restrict__ M, float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  float s = 0.f;
  for (int j = 0; j < cols; ++j) s += M[(long)j * rows + i];
  out[i] = s;
}

// per sample s (block): L_s = ||Y_s - T_s||^2 / ||T_s||^2, dY_s = 2 (Y_s - T_s) / ||T_s||^2 / B
__global__ __launch_bounds__(256) void k_relloss(int n, int B, const float* __restrict__ Y,
                                                 const float* __restrict__ T, float* __restrict__ dY,
                                                 double* __restrict__ loss) {
  __shared__ double sh[8];
  const int s = blockIdx.x;
  const float* y = Y + (long)s * n;
  const float* t = T + (long)s * n;
  double ee = 0.0, tt = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double d = (double)y[i] - (double)t[i];
    ee += d * d;
    tt += (double)t[i] * t[i];
  }
  ee = block_sum_d(ee, sh);
  tt = block_sum_d(tt, sh);
  const double inv = tt > 0.0 ? 1.0 / tt : 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    dY[(long)s * n + i] = (float)(2.0 * ((double)y[i] - (double)t[i]) * inv / B);
  if (threadIdx.x == 0) atomicAdd(loss, ee * inv / B);
}

// Adam on FP32 masters; the FP16 working copy follows
__global__ void k_adam(long n, float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, float lr, float c1, float c2, unsigned short* __restrict__ w16) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gi = g[e];
  const float a = 0.9f * m1[e] + 0.1f * gi;
  const float b = 0.999f * m2[e] + 0.001f * gi * gi;
  m1[e] = a;
  m2[e] = b;
  const float v = w[e] - lr * (a / c1) / (sqrtf(b / c2) + 1e-8f);
  w[e] = v;
  w16[e] = __half_as_ushort(__float2half(v));
}

__global__ void k_to_half(long n, const float* __restrict__ w, unsigned short* __restrict__ w16) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) w16[e] = __half_as_ushort(__float2half(w[e]));
}

// one block per (component c, column j): r = R[c*ns*ld + i*ld + j]
__global__ __launch_bounds__(256) void k_collect(int ns, int ncols, const double* __restrict__ R,
                                                 const double* __restrict__ Z, long ld,
                                                 const double* __restrict__ Dinv, float* __restrict__ X,
                                                 float* __restrict__ T) {
  __shared__ double sh[8];
  const int c = blockIdx.x / ncols, j = blockIdx.x % ncols;
  const double* r = R + (long)c * ns * ld + j;
  const double* z = Z + (long)c * ns * ld + j;
  double nn = 0.0;
  for (int i = threadIdx.x; i < ns; i += blockDim.x) nn += r[(long)i * ld] * r[(long)i * ld];
  nn = block_sum_d(nn, sh);
  const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
  float* x = X + (long)blockIdx.x * ns;
  float* t = T + (long)blockIdx.x * ns;
  for (int i = threadIdx.x; i < ns; i += blockDim.x) {
    const double ri = r[(long)i * ld];
    x[i] = (float)(ri * inv);
    t[i] = (float)((z[(long)i * ld] - Dinv[i] * ri) * inv);
  }
}

// colnorm[j] = ||R[:, j]||, colinv[j] = 1 / colnorm[j] (0 for a zero column)
__global__ __launch_bounds__(256) void k_colnorm(int ns, const double* __restrict__ R, long ld, float* __restrict__ nrm,
                                                 float* __restrict__ inv) {
  __shared__ double sh[8];
  const int j = blockIdx.x;
  double nn = 0.0;
  for (int i = threadIdx.x; i < ns; i += blockDim.x) nn += R[(long)i * ld + j] * R[(long)i * ld + j];
  nn = block_sum_d(nn, sh);
  if (threadIdx.x == 0) {
    const double v = sqrt(nn);
    nrm[j] = (float)v;
    inv[j] = v > 0.0 ? (float)(1.0 / v) : 0.f;
  }
}

// Z[i*ld + j] = Dinv[i] R[i*ld + j] + nrm[j] (Y[j*ns + i] + b3[i])
__global__ void k_mlp_out(int ns, int ncols, const double* __restrict__ R, double* __restrict__ Z, long ld,
                          const double* __restrict__ Dinv, const float* __restrict__ Y, const float* __restrict__ b3,
                          const float* __restrict__ nrm) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)ns * ncols) return;
  const int i = e / ncols, j = e % ncols;
  Z[(long)i * ld + j] = Dinv[i] * R[(long)i * ld + j] + (double)nrm[j] * ((double)Y[(long)j * ns + i] + b3[i]);
}

__global__ void k_gather_samples(int n, int B, const long* __restrict__ idx, const float* __restrict__ X,
                                 const float* __restrict__ T, float* __restrict__ Xb, float* __restrict__ Tb) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * B) return;
  const long s = e / n, i = e % n;
  Xb[e] = X[idx[s] * n + i];
  Tb[e] = T[idx[s] * n + i];
}

float* grow(float*& p, size_t& have, size_t need) {
  if (need > have) {
    if (p) (void)hipFree(p);
    p = nullptr;
    MLP_HIP(hipMalloc(&p, need * sizeof(float)));
    have = need;
  }
  return p;
}

}  // namespace

Mlp::~Mlp() {
  for (void* p : {(void*)master, (void*)grad, (void*)m1, (void*)m2, (void*)w16, (void*)X, (void*)T, (void*)act,
                  (void*)dscal})
    if (p) (void)hipFree(p);
}

Mlp* mlp_create(hipStream_t s, int n, int w, long cap, unsigned seed) {
  if (n < 1 || w < 1 || cap < 0) throw std::runtime_error("invalid network size");
  Mlp* m = new Mlp;
  m->s = s;
  m->n = n;
  m->w = w;
  m->cap = cap;
  m->off_W1 = 0;
  m->off_b1 = m->off_W1 + (size_t)w * n;
  m->off_W2 = m->off_b1 + w;
  m->off_b2 = m->off_W2 + (size_t)w * w;
  m->off_W3 = m->off_b2 + w;
  m->off_b3 = m->off_W3 + (size_t)n * w;
  m->nparam = m->off_b3 + n;
  try {
    MLP_HIP(hipMalloc(&m->master, m->nparam * sizeof(float)));
    MLP_HIP(hipMalloc(&m->grad, m->nparam * sizeof(float)));
    MLP_HIP(hipMalloc(&m->m1, m->nparam * sizeof(float)));
    MLP_HIP(hipMalloc(&m->m2, m->nparam * sizeof(float)));
    MLP_HIP(hipMalloc(&m->w16, m->nparam * sizeof(unsigned short)));
    MLP_HIP(hipMalloc(&m->dscal, 16 * sizeof(double)));
    if (cap > 0) {
      MLP_HIP(hipMalloc(&m->X, (size_t)cap * n * sizeof(float)));
      MLP_HIP(hipMalloc(&m->T, (size_t)cap * n * sizeof(float)));
    }
    // He-scaled normal weights, zero biases
    std::vector<float> h(m->nparam, 0.f);
    std::mt19937_64 g(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    for (size_t i = 0; i < (size_t)w * n; ++i) h[m->off_W1 + i] = (float)(nd(g) * std::sqrt(2.0 / n));
    for (size_t i = 0; i < (size_t)w * w; ++i) h[m->off_W2 + i] = (float)(nd(g) * std::sqrt(2.0 / w));
    for (size_t i = 0; i < (size_t)n * w; ++i) h[m->off_W3 + i] = (float)(nd(g) * std::sqrt(1.0 / w));
    mlp_set_params(*m, h.data());
  } catch (...) {
    delete m;
    throw;
  }
  return m;
}

void mlp_set_params(Mlp& m, const float* host) {
  MLP_HIP(hipMemcpyAsync(m.master, host, m.nparam * sizeof(float), hipMemcpyHostToDevice, m.s));
  hipLaunchKernelGGL(k_to_half, dim3(cdivu(m.nparam, 256)), dim3(256), 0, m.s, (long)m.nparam, m.master, m.w16);
  MLP_HIP(hipMemsetAsync(m.m1, 0, m.nparam * sizeof(float), m.s));
  MLP_HIP(hipMemsetAsync(m.m2, 0, m.nparam * sizeof(float), m.s));
  m.adam_t = 0;
  MLP_HIP(hipStreamSynchronize(m.s));
}

void mlp_get_params(const Mlp& m, float* host) {
  MLP_HIP(hipMemcpyAsync(host, m.master, m.nparam * sizeof(float), hipMemcpyDeviceToHost, m.s));
  MLP_HIP(hipStreamSynchronize(m.s));
}

namespace {
// activations for B samples: Z1/H1 (w x B), Z2/H2 (w x B), Y (n x B), dY,
// dH (w x B, two), plus batch inputs / targets (n x B each)
struct Acts {
  float *H1, *H2, *Y, *dY, *dA, *dB, *Xb, *Tb;
};
Acts acts(Mlp& m, int B) {
  const size_t w = m.w, n = m.n;
  const size_t need = (size_t)B * (4 * w + 4 * n);
  float* a = grow(m.act, m.act_n, need);
  Acts r;
  r.H1 = a;
  r.H2 = r.H1 + w * B;
  r.dA = r.H2 + w * B;
  r.dB = r.dA + w * B;
  r.Y = r.dB + w * B;
  r.dY = r.Y + n * B;
  r.Xb = r.dY + n * B;
  r.Tb = r.Xb + n * B;
  return r;
}

// forward on sample-major inputs X (column s at X + s*n) into a.H1, a.H2, a.Y.
// f16: every product on the FP16 matrix cores (inputs scaled by colscale and
// rounded to FP16 as they are staged, activations rounded likewise), as the
// solver's correction runs; otherwise FP16 weights widened to FP32 against
// FP32 activations (training, whose gradients need the wider operands).
template <class TX>
void forward(Mlp& m, const TX* X, long sXk, long sXj, const float* colscale, int B, Acts& a, bool f16) {
  const int n = m.n, w = m.w;
  const unsigned short* W1 = m.w16 + m.off_W1;
  const unsigned short* W2 = m.w16 + m.off_W2;
  const unsigned short* W3 = m.w16 + m.off_W3;
  if (f16) {
    mgemm_h(m.s, w, B, n, 1.f, W1, (long)n, 1L, X, sXk, sXj, colscale, 0.f, a.H1, 1L, (long)w);
    hipLaunchKernelGGL(k_bias_act, dim3(cdivu((long)w * B, 256)), dim3(256), 0, m.s, w, B, a.H1,
                       m.master + m.off_b1, nullptr, 1);
    mgemm_h(m.s, w, B, w, 1.f, W2, (long)w, 1L, a.H1, 1L, (long)w, nullptr, 0.f, a.H2, 1L, (long)w);
    hipLaunchKernelGGL(k_bias_act, dim3(cdivu((long)w * B, 256)), dim3(256), 0, m.s, w, B, a.H2,
                       m.master + m.off_b2, nullptr, 1);
    mgemm_h(m.s, n, B, w, 1.f, W3, (long)w, 1L, a.H2, 1L, (long)w, nullptr, 0.f, a.Y, 1L, (long)n);
    return;
  }
  mgemm(m.s, w, B, n, 1.f, W1, (long)n, 1L, X, sXk, sXj, 0.f, a.H1, 1L, (long)w);
  hipLaunchKernelGGL(k_bias_act, dim3(cdivu((long)w * B, 256)), dim3(256), 0, m.s, w, B, a.H1, m.master + m.off_b1,
                     colscale, 1);
  mgemm(m.s, w, B, w, 1.f, W2, (long)w, 1L, a.H1, 1L, (long)w, 0.f, a.H2, 1L, (long)w);
  hipLaunchKernelGGL(k_bias_act, dim3(cdivu((long)w * B, 256)), dim3(256), 0, m.s, w, B, a.H2, m.master + m.off_b2,
                     nullptr, 1);
  mgemm(m.s, n, B, w, 1.f, W3, (long)w, 1L, a.H2, 1L, (long)w, 0.f, a.Y, 1L, (long)n);
}

// loss and gradients for the batch in a.Xb / a.Tb; returns the loss (syncs)
double loss_grad(Mlp& m, int B, Acts& a) {
  const int n = m.n, w = m.w;
  forward(m, a.Xb, 1L, (long)n, nullptr, B, a, false);
  hipLaunchKernelGGL(k_bias_act, dim3(cdivu((long)n * B, 256)), dim3(256), 0, m.s, n, B, a.Y, m.master + m.off_b3,
                     nullptr, 0);
  MLP_HIP(hipMemsetAsync(m.dscal, 0, sizeof(double), m.s));
  hipLaunchKernelGGL(k_relloss, dim3(B), dim3(256), 0, m.s, n, B, a.Y, a.Tb, a.dY, m.dscal);
  float* g = m.grad;
  const unsigned short* W2 = m.w16 + m.off_W2;
  const unsigned short* W3 = m.w16 + m.off_W3;
  // layer 3
  mgemm(m.s, n, w, B, 1.f, a.dY, 1L, (long)n, a.H2, (long)w, 1L, 0.f, g + m.off_W3, (long)w, 1L);
  hipLaunchKernelGGL(k_rowsum, dim3(cdivu(n, 256)), dim3(256), 0, m.s, n, B, a.dY, g + m.off_b3);
  mgemm(m.s, w, B, n, 1.f, W3, 1L, (long)w, a.dY, 1L, (long)n, 0.f, a.dA, 1L, (long)w);
  hipLaunchKernelGGL(k_relu_bwd, dim3(cdivu((long)w * B, 256)), dim3(256), 0, m.s, (long)w * B, a.dA, a.H2);
  // layer 2
  mgemm(m.s, w, w, B, 1.f, a.dA, 1L, (long)w, a.H1, (long)w, 1L, 0.f, g + m.off_W2, (long)w, 1L);
  hipLaunchKernelGGL(k_rowsum, dim3(cdivu(w, 256)), dim3(256), 0, m.s, w, B, a.dA, g + m.off_b2);
  mgemm(m.s, w, B, w, 1.f, W2, 1L, (long)w, a.dA, 1L, (long)w, 0.f, a.dB, 1L, (long)w);
  hipLaunchKernelGGL(k_relu_bwd, dim3(cdivu((long)w * B, 256)), dim3(256), 0, m.s, (long)w * B, a.dB, a.H1);
  // layer 1
  mgemm(m.s, w, n, B, 1.f, a.dB, 1L, (long)w, a.Xb, (long)n, 1L, 0.f, g + m.off_W1, (long)n, 1L);
  hipLaunchKernelGGL(k_rowsum, dim3(cdivu(w, 256)), dim3(256), 0, m.s, w, B, a.dB, g + m.off_b1);
  double L = 0.0;
  MLP_HIP(hipMemcpyAsync(&L, m.dscal, sizeof(double), hipMemcpyDeviceToHost, m.s));
  MLP_HIP(hipStreamSynchronize(m.s));
  return L;
}
}  // namespace

void mlp_forward_host(Mlp& m, const float* Xh, int B, float* Yh, bool f16) {
  if (B < 1) return;
  Acts a = acts(m, B);
  MLP_HIP(hipMemcpyAsync(a.Xb, Xh, (size_t)B * m.n * sizeof(float), hipMemcpyHostToDevice, m.s));
  forward(m, a.Xb, 1L, (long)m.n, nullptr, B, a, f16);
  hipLaunchKernelGGL(k_bias_act, dim3(cdivu((long)m.n * B, 256)), dim3(256), 0, m.s, m.n, B, a.Y,
                     m.master + m.off_b3, nullptr, 0);
  MLP_HIP(hipMemcpyAsync(Yh, a.Y, (size_t)B * m.n * sizeof(float), hipMemcpyDeviceToHost, m.s));
  MLP_HIP(hipStreamSynchronize(m.s));
}

double mlp_loss_grad_host(Mlp& m, const float* Xh, const float* Th, int B, float* gh) {
  if (B < 1) throw std::runtime_error("empty batch");
  Acts a = acts(m, B);
  MLP_HIP(hipMemcpyAsync(a.Xb, Xh, (size_t)B * m.n * sizeof(float), hipMemcpyHostToDevice, m.s));
  MLP_HIP(hipMemcpyAsync(a.Tb, Th, (size_t)B * m.n * sizeof(float), hipMemcpyHostToDevice, m.s));
  double L = loss_grad(m, B, a);
  if (gh) {
    MLP_HIP(hipMemcpyAsync(gh, m.grad, m.nparam * sizeof(float), hipMemcpyDeviceToHost, m.s));
    MLP_HIP(hipStreamSynchronize(m.s));
  }
  return L;
}

void mlp_train(Mlp& m, int steps, int B, double lr, unsigned seed, double* losses) {
  if (m.count < 1) throw std::runtime_error("no training pairs collected");
  if (B < 1) throw std::runtime_error("empty batch");
  std::mt19937_64 g(seed);
  std::uniform_int_distribution<long> pick(0, m.count - 1);
  // batch >= count: every step is the full batch of all pairs, in order
  const bool full = B >= m.count;
  if (full) B = (int)m.count;
  long* didx = nullptr;
  MLP_HIP(hipMalloc(&didx, (size_t)B * sizeof(long)));
  std::vector<long> idx(B);
  try {
    for (int st = 0; st < steps; ++st) {
      Acts a = acts(m, B);
      for (int i = 0; i < B; ++i) idx[i] = full ? i : pick(g);
      MLP_HIP(hipMemcpyAsync(didx, idx.data(), (size_t)B * sizeof(long), hipMemcpyHostToDevice, m.s));
      hipLaunchKernelGGL(k_gather_samples, dim3(cdivu((long)m.n * B, 256)), dim3(256), 0, m.s, m.n, B, didx, m.X, m.T,
                         a.Xb, a.Tb);
      const double L = loss_grad(m, B, a);
      if (losses) losses[st] = L;
      ++m.adam_t;
      const float c1 = 1.f - std::pow(0.9f, (float)m.adam_t), c2 = 1.f - std::pow(0.999f, (float)m.adam_t);
      hipLaunchKernelGGL(k_adam, dim3(cdivu(m.nparam, 256)), dim3(256), 0, m.s, (long)m.nparam, m.master, m.grad,
                         m.m1, m.m2, (float)lr, c1, c2, m.w16);
    }
    MLP_HIP(hipStreamSynchronize(m.s));
  } catch (...) {
    (void)hipFree(didx);
    throw;
  }
  (void)hipFree(didx);
}

long mlp_add_pairs(Mlp& m, const float* Xh, const float* Th, long count) {
  const long k = std::max(0L, std::min(count, m.cap - m.count));
  if (k > 0) {
    MLP_HIP(hipMemcpyAsync(m.X + m.count * (long)m.n, Xh, (size_t)k * m.n * sizeof(float), hipMemcpyHostToDevice, m.s));
    MLP_HIP(hipMemcpyAsync(m.T + m.count * (long)m.n, Th, (size_t)k * m.n * sizeof(float), hipMemcpyHostToDevice, m.s));
    MLP_HIP(hipStreamSynchronize(m.s));
    m.count += k;
  }
  return k;
}

void mlp_collect(Mlp& m, int ns, int ncomp, int ncols, const double* R, const double* Z, long ld,
                 const double* Dinv) {
  if (ns != m.n) throw std::runtime_error("network size does not match the spatial solve");
  const long want = (long)ncomp * ncols;
  if (m.count + want > m.cap) return;   // buffer full: keep what was collected
  hipLaunchKernelGGL(k_collect, dim3((unsigned)want), dim3(256), 0, m.s, ns, ncols, R, Z, ld, Dinv,
                     m.X + m.count * (long)ns, m.T + m.count * (long)ns);
  m.count += want;
}

void mlp_apply(Mlp& m, int ns, int ncomp, int ncols, const double* R, double* Z, long ld, const double* Dinv) {
  if (ns != m.n) throw std::runtime_error("network size does not match the spatial solve");
  if (ncols < 1) return;
  Acts a = acts(m, ncols);
  float* nrm = a.dY;            // 2 * ncols floats of the (unused here) gradient space
  float* inv = a.dY + ncols;
  for (int c = 0; c < ncomp; ++c) {
    const double* Rc = R + (long)c * ns * ld;
    double* Zc = Z + (long)c * ns * ld;
    hipLaunchKernelGGL(k_colnorm, dim3(ncols), dim3(256), 0, m.s, ns, Rc, ld, nrm, inv);
    forward(m, Rc, ld, 1L, inv, ncols, a, true);
    hipLaunchKernelGGL(k_mlp_out, dim3(cdivu((long)ns * ncols, 256)), dim3(256), 0, m.s, ns, ncols, Rc, Zc, ld, Dinv,
                       a.Y, m.master + m.off_b3, nrm);
  }
}

}  // namespace sgtt
