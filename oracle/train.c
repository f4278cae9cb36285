/* Oracle training: double-precision loss, gradient by the chain rule, Adam.
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * The learned heuristic is fitted to distance labels; the paper's design
 * objective asks for a large mean h without over-estimating (h_M <= h*),
 * which motivates the optional asymmetric loss: squared error weighted by
 * alpha when the prediction exceeds the label.
 *   L = (1/n) sum_b w_b (y_b - t_b)^2,  w_b = alpha if (asym and y_b > t_b) else 1
 * Network and tensor order as in mlp.c (file order).  ReLU'(z) is taken as 1
 * for z > 0 and 0 otherwise, i.e. the gradient flows where the stored
 * activation is positive.
 * Adam (Kingma & Ba 2015): m <- b1 m + (1-b1) g; v <- b2 v + (1-b2) g^2;
 * w <- w - lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "orc.h"

#define MAXT ORC_MAXT

int orc_net_param_count(const orc_net* m) {
    int64_t n = 0;
    for (int t = 0; t < m->nt; t++) n += (int64_t)m->rows[t] * m->cols[t];
    return (int)n;
}

/* Copy all parameters into / out of a flat array (file order). */
void orc_net_get_params(const orc_net* m, double* flat) {
    for (int t = 0; t < m->nt; t++) {
        size_t c = (size_t)m->rows[t] * m->cols[t];
        memcpy(flat, m->T[t], c * sizeof(double));
        flat += c;
    }
}

void orc_net_set_params(orc_net* m, const double* flat) {
    for (int t = 0; t < m->nt; t++) {
        size_t c = (size_t)m->rows[t] * m->cols[t];
        memcpy(m->T[t], flat, c * sizeof(double));
        flat += c;
    }
}

/* Loss over a batch and its gradient (grads: flat, file order, same size as the
 * parameters; overwritten).  Regression nets only (one output). */
double orc_train_grad(const orc_net* m, const uint8_t* states, int64_t n, const double* labels, int asym,
                      double alpha, double* grads, double* y_out) {
    int np = orc_net_param_count(m);
    memset(grads, 0, (size_t)np * sizeof(double));
    double* G[MAXT];
    {
        double* p = grads;
        for (int t = 0; t < m->nt; t++) { G[t] = p; p += (size_t)m->rows[t] * m->cols[t]; }
    }
    int maxw = 1;
    for (int i = 0; i < m->n_dense; i++) if (m->dims[i] > maxw) maxw = m->dims[i];
    const int nd = m->n_dense, nr = m->n_res, H = m->dims[nd - 1];
    /* saved activations: x[0..nd-1] (dense outputs), t[r], xr[r] (block outputs) */
    int nsave = nd + 2 * nr;
    double* A = (double*)malloc((size_t)nsave * maxw * sizeof(double));
    double* g = (double*)malloc((size_t)maxw * sizeof(double));
    double* g2 = (double*)malloc((size_t)maxw * sizeof(double));
    double* gt = (double*)malloc((size_t)maxw * sizeof(double));
    double loss = 0.0;
    for (int64_t b = 0; b < n; b++) {
        const uint8_t* s = states + b * m->P;
        /* ---- forward, saving post-ReLU activations */
        double* x0 = A;
        for (int j = 0; j < m->dims[0]; j++) x0[j] = m->T[1][j];
        for (int p = 0; p < m->P; p++) {
            int row = p * m->S + s[p];
            for (int j = 0; j < m->dims[0]; j++) x0[j] += m->T[0][(size_t)row * m->dims[0] + j];
        }
        for (int j = 0; j < m->dims[0]; j++) if (x0[j] < 0) x0[j] = 0;
        int ti = 2;
        for (int i = 1; i < nd; i++) {
            double* xi = A + (size_t)i * maxw;
            double* xp = A + (size_t)(i - 1) * maxw;
            int K = m->dims[i - 1], N = m->dims[i];
            for (int j = 0; j < N; j++) {
                double acc = m->T[ti + 1][j];
                for (int k = 0; k < K; k++) acc += xp[k] * m->T[ti][(size_t)k * N + j];
                xi[j] = acc > 0 ? acc : 0;
            }
            ti += 2;
        }
        double* xin = A + (size_t)(nd - 1) * maxw;
        for (int r = 0; r < nr; r++) {
            double* tr = A + (size_t)(nd + 2 * r) * maxw;
            double* xo = A + (size_t)(nd + 2 * r + 1) * maxw;
            for (int j = 0; j < H; j++) {
                double acc = m->T[ti + 1][j];
                for (int k = 0; k < H; k++) acc += xin[k] * m->T[ti][(size_t)k * H + j];
                tr[j] = acc > 0 ? acc : 0;
            }
            for (int j = 0; j < H; j++) {
                double acc = m->T[ti + 3][j] + xin[j];
                for (int k = 0; k < H; k++) acc += tr[k] * m->T[ti + 2][(size_t)k * H + j];
                xo[j] = acc > 0 ? acc : 0;
            }
            xin = xo;
            ti += 4;
        }
        const int th = ti; /* head tensor index */
        double y = m->T[th + 1][0];
        for (int k = 0; k < H; k++) y += xin[k] * m->T[th][k];
        if (y_out) y_out[b] = y;
        double d = y - labels[b];
        double w = (asym && d > 0) ? alpha : 1.0;
        loss += w * d * d / (double)n;
        double dy = 2.0 * w * d / (double)n;
        /* ---- backward */
        G[th + 1][0] += dy;
        for (int k = 0; k < H; k++) {
            G[th][k] += xin[k] * dy;
            g[k] = (xin[k] > 0) ? dy * m->T[th][k] : 0.0; /* gradient w.r.t. the pre-activation of xin */
        }
        ti = th;
        for (int r = nr - 1; r >= 0; r--) {
            ti -= 4;
            double* tr = A + (size_t)(nd + 2 * r) * maxw;
            double* xi = (r == 0) ? A + (size_t)(nd - 1) * maxw : A + (size_t)(nd + 2 * (r - 1) + 1) * maxw;
            /* g = dL/d(pre-activation of the block output) = gu */
            for (int j = 0; j < H; j++) G[ti + 3][j] += g[j];
            for (int k = 0; k < H; k++) {
                double acc = 0.0;
                for (int j = 0; j < H; j++) {
                    G[ti + 2][(size_t)k * H + j] += tr[k] * g[j];
                    acc += g[j] * m->T[ti + 2][(size_t)k * H + j];
                }
                gt[k] = tr[k] > 0 ? acc : 0.0;
            }
            for (int j = 0; j < H; j++) G[ti + 1][j] += gt[j];
            for (int k = 0; k < H; k++) {
                double acc = g[k]; /* identity path of the residual */
                for (int j = 0; j < H; j++) {
                    G[ti][(size_t)k * H + j] += xi[k] * gt[j];
                    acc += gt[j] * m->T[ti][(size_t)k * H + j];
                }
                g2[k] = xi[k] > 0 ? acc : 0.0;
            }
            memcpy(g, g2, (size_t)H * sizeof(double));
        }
        for (int i = nd - 1; i >= 1; i--) {
            ti -= 2;
            double* xp = A + (size_t)(i - 1) * maxw;
            int K = m->dims[i - 1], N = m->dims[i];
            for (int j = 0; j < N; j++) G[ti + 1][j] += g[j];
            for (int k = 0; k < K; k++) {
                double acc = 0.0;
                for (int j = 0; j < N; j++) {
                    G[ti][(size_t)k * N + j] += xp[k] * g[j];
                    acc += g[j] * m->T[ti][(size_t)k * N + j];
                }
                g2[k] = xp[k] > 0 ? acc : 0.0;
            }
            memcpy(g, g2, (size_t)K * sizeof(double));
        }
        /* layer 1: the one-hot input selects P rows */
        for (int j = 0; j < m->dims[0]; j++) G[1][j] += g[j];
        for (int p = 0; p < m->P; p++) {
            int row = p * m->S + s[p];
            for (int j = 0; j < m->dims[0]; j++) G[0][(size_t)row * m->dims[0] + j] += g[j];
        }
    }
    free(A); free(g); free(g2); free(gt);
    return loss;
}

void orc_adam_step(double* w, const double* g, double* mo, double* vo, int64_t n, double lr, double b1, double b2,
                   double eps, int t) {
    double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
    for (int64_t i = 0; i < n; i++) {
        mo[i] = b1 * mo[i] + (1.0 - b1) * g[i];
        vo[i] = b2 * vo[i] + (1.0 - b2) * g[i] * g[i];
        w[i] -= lr * (mo[i] / c1) / (sqrt(vo[i] / c2) + eps);
    }
}
