// Learned correction of the mean spatial solve in the inner preconditioner
// (eq. 5.23): z = D^-1 r + ||r|| * MLP(r / ||r||) with D = diag(F_avg) and a
// three-layer perceptron n -> w -> w -> n (ReLU), FP16 weights, FP32
// activations and accumulation on the matrix cores, trained on the device
// with hand-written backward kernels and Adam on FP32 master weights.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <vector>

namespace sgtt {

struct Mlp {
  hipStream_t s = nullptr;
  int n = 0, w = 0;
  long cap = 0, count = 0;      // collected training pairs
  long adam_t = 0;
  // FP32 master parameters [W1 (w x n), b1 (w), W2 (w x w), b2 (w), W3 (n x w), b3 (n)]
  float* master = nullptr;
  float* grad = nullptr;
  float* m1 = nullptr;
  float* m2 = nullptr;
  unsigned short* w16 = nullptr;   // FP16 working copies of W1, W2, W3 (same offsets as master)
  size_t nparam = 0;
  size_t off_W1 = 0, off_b1 = 0, off_W2 = 0, off_b2 = 0, off_W3 = 0, off_b3 = 0;
  // training pairs: sample s occupies [s*n, (s+1)*n) of X and T
  float* X = nullptr;
  float* T = nullptr;
  // activations / workspace for a batch (grown on demand)
  float* act = nullptr;
  size_t act_n = 0;
  double* dscal = nullptr;         // device loss accumulator
  int uses = 0;                    // systems holding it (attached or collecting)
  ~Mlp();
};

Mlp* mlp_create(hipStream_t s, int n, int w, long cap, unsigned seed);
void mlp_set_params(Mlp& m, const float* host);
void mlp_get_params(const Mlp& m, float* host);
// Y (n x B, sample-major: column s at Y + s*n) = MLP(X) for inputs in the same
// layout; f16: the products on FP16 matrix cores with FP16 operands (the
// form the solver's correction uses), else FP32 operands (training's form)
void mlp_forward_host(Mlp& m, const float* Xh, int B, float* Yh, bool f16);
// loss and gradients (FP32) for host inputs / targets; grads in parameter order
double mlp_loss_grad_host(Mlp& m, const float* Xh, const float* Th, int B, float* gh);
// Adam training on the collected pairs: steps minibatches of B pairs
void mlp_train(Mlp& m, int steps, int B, double lr, unsigned seed, double* losses);
// Append host pairs (column s at Xh + s*n); returns how many fit.
long mlp_add_pairs(Mlp& m, const float* Xh, const float* Th, long count);
// Record pairs from one mean solve: for every component c < ncomp and column
// j, r = R[c*ns*ld + i*ld + j] and z = Z[...] (exact F_avg^-1 r); stores
// x = r/||r||, t = (z - Dinv r)/||r||.  Stops when the buffer is full.
void mlp_collect(Mlp& m, int ns, int ncomp, int ncols, const double* R, const double* Z, long ld,
                 const double* Dinv);
// Z = Dinv R + ||r|| MLP(r / ||r||) for every component and column (same
// layout as mlp_collect).
void mlp_apply(Mlp& m, int ns, int ncomp, int ncols, const double* R, double* Z, long ld, const double* Dinv);

}  // namespace sgtt
