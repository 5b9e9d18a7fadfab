// FP64 CPU oracle of the block-visibility prefetch predictor: a ReLU MLP
// whose weights are rounded to bfloat16 (round to nearest even), evaluated
// and differentiated in double precision, with a binary cross-entropy-with-
// logits loss averaged over the valid outputs.
//
// TEST INFRASTRUCTURE ONLY; shares no code with the product library.
//
// Layer l maps in_l -> out_l: a_{l+1} = relu(W_l a_l + b_l) for hidden
// layers, z = W_L a_L + b_L for the output (logits).  W_l is stored
// row-major [out_l][in_l].  Loss over the batch and the valid outputs:
//   l(z, y) = max(z, 0) - z y + log(1 + exp(-|z|)),  mean over (sample, valid output).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

// bfloat16 rounding of a float: keep the upper 16 bits of the IEEE single,
// rounding the lower 16 to nearest, ties to even.
double bf16_round_one(double x) {
  const float f = (float)x;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return x;   // inf / nan untouched
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  u &= 0xffff0000u;
  float r;
  std::memcpy(&r, &u, 4);
  return (double)r;
}

}  // namespace

extern "C" {

void orc_bf16_round(const double* x, int64_t n, double* y) {
  for (int64_t i = 0; i < n; ++i) y[i] = bf16_round_one(x[i]);
}

// dims[0..L]: layer widths (dims[0] = input, dims[L] = output).  W[l], b[l]
// for l < L.  x [batch][dims[0]] -> logits [batch][dims[L]].  Weights are
// used as given (round them with orc_bf16_round first).
void orc_mlp_forward(const double* x, int batch, const int32_t* dims, int L, double** W, double** b,
                     double* logits) {
  for (int s = 0; s < batch; ++s) {
    std::vector<double> a(x + (int64_t)s * dims[0], x + (int64_t)(s + 1) * dims[0]);
    for (int l = 0; l < L; ++l) {
      std::vector<double> z(dims[l + 1]);
      for (int o = 0; o < dims[l + 1]; ++o) {
        double acc = b[l][o];
        for (int i = 0; i < dims[l]; ++i) acc += W[l][(int64_t)o * dims[l] + i] * a[i];
        z[o] = (l + 1 < L) ? (acc > 0 ? acc : 0.0) : acc;
      }
      a.swap(z);
    }
    std::memcpy(logits + (int64_t)s * dims[L], a.data(), sizeof(double) * dims[L]);
  }
}

// Loss and gradients.  labels[s][o] in {0,1} (u8), valid[o] in {0,1} (u8)
// marks the outputs that count.  Writes the mean loss and dW[l], db[l]
// (overwritten).
void orc_mlp_loss_backward(const double* x, int batch, const int32_t* dims, int L, double** W, double** b,
                           const uint8_t* labels, const uint8_t* valid, int unused, double* loss, double** dW,
                           double** db) {
  (void)unused;
  const int nout = dims[L];
  int64_t nvalid = 0;
  for (int o = 0; o < nout; ++o) nvalid += valid[o] ? 1 : 0;
  const double denom = (double)batch * (double)(nvalid > 0 ? nvalid : 1);
  for (int l = 0; l < L; ++l) {
    std::memset(dW[l], 0, sizeof(double) * (size_t)dims[l] * dims[l + 1]);
    std::memset(db[l], 0, sizeof(double) * dims[l + 1]);
  }
  double total = 0;
  for (int s = 0; s < batch; ++s) {
    // forward, keeping every layer's input and pre-activation
    std::vector<std::vector<double>> act(L + 1), pre(L);
    act[0].assign(x + (int64_t)s * dims[0], x + (int64_t)(s + 1) * dims[0]);
    for (int l = 0; l < L; ++l) {
      pre[l].resize(dims[l + 1]);
      act[l + 1].resize(dims[l + 1]);
      for (int o = 0; o < dims[l + 1]; ++o) {
        double acc = b[l][o];
        for (int i = 0; i < dims[l]; ++i) acc += W[l][(int64_t)o * dims[l] + i] * act[l][i];
        pre[l][o] = acc;
        act[l + 1][o] = (l + 1 < L) ? (acc > 0 ? acc : 0.0) : acc;
      }
    }
    // BCE with logits and its gradient
    std::vector<double> g(nout, 0.0);
    for (int o = 0; o < nout; ++o) {
      if (!valid[o]) continue;
      const double z = act[L][o], y = labels[(int64_t)s * nout + o] ? 1.0 : 0.0;
      total += std::max(z, 0.0) - z * y + std::log1p(std::exp(-std::fabs(z)));
      g[o] = (1.0 / (1.0 + std::exp(-z)) - y) / denom;
    }
    // backward
    for (int l = L - 1; l >= 0; --l) {
      std::vector<double> gin(dims[l], 0.0);
      for (int o = 0; o < dims[l + 1]; ++o) {
        double go = g[o];
        if (l + 1 < L && !(pre[l][o] > 0)) go = 0.0;   // ReLU
        if (go == 0.0) continue;
        db[l][o] += go;
        for (int i = 0; i < dims[l]; ++i) {
          dW[l][(int64_t)o * dims[l] + i] += go * act[l][i];
          gin[i] += go * W[l][(int64_t)o * dims[l] + i];
        }
      }
      g.swap(gin);
    }
  }
  *loss = total / denom;
}

// One Adam step (no weight decay) on n parameters, FP64, in place:
//   m <- b1 m + (1-b1) g,  v <- b2 v + (1-b2) g^2,
//   p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
void orc_mlp_adam(double* p, const double* g, double* m, double* v, int64_t n, int64_t t, double lr, double b1,
                  double b2, double eps) {
  const double c1 = 1.0 - std::pow(b1, (double)t), c2 = 1.0 - std::pow(b2, (double)t);
  for (int64_t i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    p[i] -= lr * (m[i] / c1) / (std::sqrt(v[i] / c2) + eps);
  }
}

}  // extern "C"
