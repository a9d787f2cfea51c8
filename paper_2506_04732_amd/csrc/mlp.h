// Learned warm start: network, training, fitting loss, packing.  See mlp.hip.
#pragma once
#include <vector>

#include "solver.h"

namespace t2s2 {

struct Mlp {
  std::vector<int> w;          // widths w_0 .. w_L
  long nparam = 0;
  float* params = nullptr;     // per layer: W_k (w_{k+1} x w_k row-major), b_k
  float* grad = nullptr;       // gradient of the last backward pass
  float* m = nullptr;          // Adam moments
  float* v = nullptr;
  unsigned short* params16 = nullptr;  // BF16 copy for inference
  bool bf16_valid = false;
  int t = 0;                   // Adam steps taken
  int last_batch = 0;          // batch of the last forward pass
  Scratch sc;
  ~Mlp();
};

long mlp_param_count(const std::vector<int>& w);
Mlp* mlp_create(const std::vector<int>& widths, unsigned long long seed);
void mlp_forward(Mlp& N, hipStream_t s, int B, const float* X, float* Y);
void mlp_backward(Mlp& N, hipStream_t s, int B, const float* X, const float* dY);
void mlp_adam(Mlp& N, hipStream_t s, float lr, float b1, float b2, float eps);
void mlp_infer_bf16(Mlp& N, hipStream_t s, int B, const float* X, float* Y);
int tt_flat_size(int d, const int* n, int r);
void tt_fit_loss(hipStream_t s, int B, int d, const int* n, int r, const float* pred, const float* target,
                 float* loss, float* dpred, float gscale);
std::vector<float> mlp_train(Mlp& N, hipStream_t s, int count, const float* X, const float* Yt, int d, const int* n,
                             int r, int epochs, int batch, float lr, unsigned long long seed);
void tt_pack(hipStream_t s, const DTT& x, int r, int canonical, float* out);
void tt_unpack(hipStream_t s, int d, const int* n, int r, const float* in, DTT& x);

}  // namespace t2s2
