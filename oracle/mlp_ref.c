/*
 * Plain CPU reference for the task cost model -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may load this library.
 * It shares no code with the GPU library.
 *
 * The cost model is a small fully connected network that maps a task's feature vector x (F
 * values) to a predicted log run time:
 *     h1 = relu(W1 x + b1)      (H1 units)
 *     h2 = relu(W2 h1 + b2)     (H2 units)
 *     y  = w3 . h2 + b3
 * trained on the mean squared error L = (1/B) sum_b (y_b - t_b)^2 with Adam
 * (Kingma & Ba, 2015: m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
 *  theta <- theta - lr * (m / (1-b1^n)) / (sqrt(v / (1-b2^n)) + eps) at step n).
 *
 * The paper itself schedules tasks dynamically and observes that load imbalance is what the task
 * formulation must absorb (Sec. 3, Sec. 4.4); the learned model only orders and bins tasks.
 *
 * Parameter vector layout (FP64 here): W1 (H1 x F, row-major), b1 (H1), W2 (H2 x H1, row-major),
 * b2 (H2), w3 (H2), b3 (1).  Plain loops, FP64 throughout, no contraction.
 */
#include <stdint.h>
#include <stdlib.h>
#include <math.h>

int64_t oracle_mlp_param_count(int64_t F, int64_t H1, int64_t H2) {
  return H1 * F + H1 + H2 * H1 + H2 + H2 + 1;
}

typedef struct {
  const double *W1, *b1, *W2, *b2, *w3, *b3;
} params_view;

static params_view view(const double* p, int64_t F, int64_t H1, int64_t H2) {
  params_view v;
  v.W1 = p;
  v.b1 = v.W1 + H1 * F;
  v.W2 = v.b1 + H1;
  v.b2 = v.W2 + H2 * H1;
  v.w3 = v.b2 + H2;
  v.b3 = v.w3 + H2;
  return v;
}

/* forward for one sample; fills z1/h1/z2/h2 (pre- and post-activation) and returns y */
static double forward_one(const params_view* v, int64_t F, int64_t H1, int64_t H2, const double* x,
                          double* z1, double* h1, double* z2, double* h2) {
  for (int64_t u = 0; u < H1; ++u) {
    double s = v->b1[u];
    for (int64_t f = 0; f < F; ++f) s += v->W1[u * F + f] * x[f];
    z1[u] = s;
    h1[u] = s > 0.0 ? s : 0.0;
  }
  for (int64_t u = 0; u < H2; ++u) {
    double s = v->b2[u];
    for (int64_t q = 0; q < H1; ++q) s += v->W2[u * H1 + q] * h1[q];
    z2[u] = s;
    h2[u] = s > 0.0 ? s : 0.0;
  }
  double y = v->b3[0];
  for (int64_t u = 0; u < H2; ++u) y += v->w3[u] * h2[u];
  return y;
}

int oracle_mlp_forward(int64_t F, int64_t H1, int64_t H2, const double* params, int64_t B,
                       const double* X, double* Y) {
  params_view v = view(params, F, H1, H2);
  double* buf = (double*)malloc((size_t)(2 * H1 + 2 * H2) * sizeof(double));
  if (!buf) return -1;
  for (int64_t b = 0; b < B; ++b)
    Y[b] = forward_one(&v, F, H1, H2, X + b * F, buf, buf + H1, buf + 2 * H1, buf + 2 * H1 + H2);
  free(buf);
  return 0;
}

/* L = (1/B) sum (y - t)^2 and its gradient with respect to every parameter (chain rule). */
double oracle_mlp_loss_grad(int64_t F, int64_t H1, int64_t H2, const double* params, int64_t B,
                            const double* X, const double* T, double* grad) {
  params_view v = view(params, F, H1, H2);
  int64_t P = oracle_mlp_param_count(F, H1, H2);
  for (int64_t q = 0; q < P; ++q) grad[q] = 0.0;
  double *gW1 = grad, *gb1 = gW1 + H1 * F, *gW2 = gb1 + H1, *gb2 = gW2 + H2 * H1;
  double *gw3 = gb2 + H2, *gb3 = gw3 + H2;
  double* buf = (double*)malloc((size_t)(3 * H1 + 3 * H2) * sizeof(double));
  if (!buf) return NAN;
  double *z1 = buf, *h1 = z1 + H1, *z2 = h1 + H1, *h2 = z2 + H2, *d2 = h2 + H2, *d1 = d2 + H2;
  double loss = 0.0;
  for (int64_t b = 0; b < B; ++b) {
    const double* x = X + b * F;
    double y = forward_one(&v, F, H1, H2, x, z1, h1, z2, h2);
    double e = y - T[b];
    loss += e * e;
    double dy = 2.0 * e / (double)B; /* dL/dy */
    gb3[0] += dy;
    for (int64_t u = 0; u < H2; ++u) {
      gw3[u] += dy * h2[u];
      d2[u] = z2[u] > 0.0 ? dy * v.w3[u] : 0.0; /* dL/dz2 */
    }
    for (int64_t q = 0; q < H1; ++q) {
      double s = 0.0;
      for (int64_t u = 0; u < H2; ++u) s += v.W2[u * H1 + q] * d2[u];
      d1[q] = z1[q] > 0.0 ? s : 0.0; /* dL/dz1 */
    }
    for (int64_t u = 0; u < H2; ++u) {
      gb2[u] += d2[u];
      for (int64_t q = 0; q < H1; ++q) gW2[u * H1 + q] += d2[u] * h1[q];
    }
    for (int64_t u = 0; u < H1; ++u) {
      gb1[u] += d1[u];
      for (int64_t f = 0; f < F; ++f) gW1[u * F + f] += d1[u] * x[f];
    }
  }
  free(buf);
  return loss / (double)B;
}

/* One Adam step (step = 1, 2, ... counts the updates made so far including this one). */
int oracle_adam_step(int64_t P, double* params, const double* grad, double* m, double* v,
                     int64_t step, double lr, double beta1, double beta2, double eps) {
  double c1 = 1.0 - pow(beta1, (double)step), c2 = 1.0 - pow(beta2, (double)step);
  for (int64_t q = 0; q < P; ++q) {
    m[q] = beta1 * m[q] + (1.0 - beta1) * grad[q];
    v[q] = beta2 * v[q] + (1.0 - beta2) * grad[q] * grad[q];
    params[q] -= lr * (m[q] / c1) / (sqrt(v[q] / c2) + eps);
  }
  return 0;
}
