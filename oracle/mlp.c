/* Oracle network: double-precision forward pass of the neural heuristic h_M,
 * its output rules, and exact emulation of reduced-precision operands.
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * The paper evaluates a neural heuristic on batches of states (CB-DFS for
 * neural heuristics; SingleGPU Batch CB-DFS), turning each generated state into
 * the network's input tensor (Subtree expansion algorithm, TensorRepresentation).
 * Input: one-hot vector of length P*S with a one at p*S + s[p] for every cell
 * (or sticker) p holding symbol s[p].
 * Network: layer 1 (one-hot input -> dims[0]), ReLU; dense layers dims[i-1] ->
 * dims[i], ReLU; n_res residual blocks x <- ReLU(x + W_b ReLU(W_a x + b_a) + b_b);
 * linear head -> n_out.
 * Output rules:
 *   regression: v = y - offset, h = floor(v) or round-half-even(v), clamped
 *     at 0, optionally min'ed with Manhattan distance (the paper's STP model
 *     builds on Manhattan distance; the regression cube model subtracts a
 *     constant, Experimental Setup);
 *   classifier: the smallest class whose cumulative softmax probability reaches
 *     q (ordered heuristic classes with an adjustable quantile, Related Work on
 *     learned admissible heuristics), or the arg-max class.
 * Reduced precision (quantised operands, double accumulation):
 *   bf16: every weight matrix and every stored activation rounded to bfloat16
 *     (round to nearest even on the float32 value);
 *   fp8:  dense and residual matrices as OCP e4m3 with one float32 scale per
 *     output column s_n = max_k |W[k][n]| / 448; stored activations as e4m3
 *     with a static power-of-two scale per tensor; layer 1 and head weights in
 *     bfloat16.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "orc.h"

#define MAXT ORC_MAXT

/* ----------------------------------------------------------- rounding */
double orc_bf16_round(double x) {
    float f = (float)x; /* round to nearest even float32 */
    if (isnan(f)) return f;
    uint32_t u;
    memcpy(&u, &f, 4);
    uint32_t lsb = (u >> 16) & 1u;
    uint32_t r = u + 0x7FFFu + lsb; /* round to nearest, ties to even */
    r &= 0xFFFF0000u;
    float o;
    memcpy(&o, &r, 4);
    return o;
}

double orc_e4m3_decode(int c) {
    int s = (c >> 7) & 1, e = (c >> 3) & 15, m = c & 7;
    if (e == 15 && m == 7) return NAN;
    double v = (e == 0) ? ldexp(m / 8.0, -6) : ldexp(1.0 + m / 8.0, e - 7);
    return s ? -v : v;
}

/* Nearest finite e4m3 value by exhaustive search over the codes, ties to the
 * even code; magnitudes beyond 448 saturate to 448. */
double orc_e4m3_round(double x) {
    if (isnan(x)) return NAN;
    double a = fabs(x);
    if (a > 448.0) a = 448.0;
    int best = 0;
    double bd = INFINITY;
    for (int c = 0; c <= 0x7E; c++) {
        double d = fabs(orc_e4m3_decode(c) - a);
        if (d < bd || (d == bd && (c & 1) == 0)) { bd = d; best = c; }
    }
    double v = orc_e4m3_decode(best);
    return x < 0 ? -v : v;
}

int orc_e4m3_encode(double x) {
    double v = orc_e4m3_round(x);
    for (int c = 0; c < 256; c++) if (orc_e4m3_decode(c) == v && (c >> 7) == (signbit(v) ? 1 : 0)) return c;
    return 0x7F;
}

void orc_bf16_round_array(const double* x, int64_t n, double* out) { for (int64_t i = 0; i < n; i++) out[i] = orc_bf16_round(x[i]); }
void orc_e4m3_round_array(const double* x, int64_t n, double* out) { for (int64_t i = 0; i < n; i++) out[i] = orc_e4m3_round(x[i]); }

/* ----------------------------------------------------------- loading */
static int dom_P(int d) { return d == ORC_STP3 ? 9 : d == ORC_STP4 ? 16 : 54; }
static int dom_S(int d) { return d == ORC_STP3 ? 9 : d == ORC_STP4 ? 16 : 6; }

void orc_net_free(orc_net* m) {
    if (!m) return;
    for (int i = 0; i < m->nt; i++) free(m->T[i]);
    free(m);
}

orc_net* orc_net_load(const char* path) {
    FILE* f = fopen(path, "rb");
    if (!f) return NULL;
    uint32_t h[5];
    orc_net* m = (orc_net*)calloc(1, sizeof(orc_net));
    if (fread(h, 4, 5, f) != 5 || h[0] != 0x31574248u || h[1] != 1 || h[4] < 1 || h[4] > 8) goto fail;
    m->domain = (int)h[2];
    m->n_in = (int)h[3];
    m->n_dense = (int)h[4];
    uint32_t d[8];
    if (fread(d, 4, (size_t)m->n_dense, f) != (size_t)m->n_dense) goto fail;
    for (int i = 0; i < m->n_dense; i++) m->dims[i] = (int)d[i];
    uint32_t t3[3];
    if (fread(t3, 4, 3, f) != 3) goto fail;
    m->n_res = (int)t3[0];
    m->n_out = (int)t3[1];
    m->head_kind = (int)t3[2];
    m->P = dom_P(m->domain);
    m->S = dom_S(m->domain);
    if (m->P * m->S != m->n_in) goto fail;
    int prev = m->n_in, nt = 0;
    for (int i = 0; i < m->n_dense; i++) {
        m->rows[nt] = prev; m->cols[nt] = m->dims[i]; nt++;
        m->rows[nt] = 1; m->cols[nt] = m->dims[i]; nt++;
        prev = m->dims[i];
    }
    for (int r = 0; r < m->n_res; r++) {
        for (int j = 0; j < 2; j++) {
            m->rows[nt] = prev; m->cols[nt] = prev; nt++;
            m->rows[nt] = 1; m->cols[nt] = prev; nt++;
        }
    }
    m->rows[nt] = prev; m->cols[nt] = m->n_out; nt++;
    m->rows[nt] = 1; m->cols[nt] = m->n_out; nt++;
    m->nt = nt;
    for (int i = 0; i < nt; i++) {
        size_t cnt = (size_t)m->rows[i] * (size_t)m->cols[i];
        float* buf = (float*)malloc(cnt * 4);
        if (fread(buf, 4, cnt, f) != cnt) { free(buf); goto fail; }
        m->T[i] = (double*)malloc(cnt * sizeof(double));
        for (size_t k = 0; k < cnt; k++) m->T[i][k] = buf[k]; /* exact widening */
        free(buf);
    }
    fclose(f);
    return m;
fail:
    fclose(f);
    orc_net_free(m);
    return NULL;
}

int orc_net_info(const orc_net* m, int* out) {
    out[0] = m->domain; out[1] = m->n_in; out[2] = m->n_dense; out[3] = m->n_res;
    out[4] = m->n_out; out[5] = m->head_kind; out[6] = m->nt;
    for (int i = 0; i < m->n_dense; i++) out[7 + i] = m->dims[i];
    return 1;
}

int orc_net_n_act(const orc_net* m) { return m->n_dense + 2 * m->n_res; }

/* ------------------------------------------------------ quantisation */
/* Effective (dequantised) weights for a precision mode: 0 none, 1 bf16, 2 fp8.
 * Tensor roles: even index < 2*n_dense-ish are weights, odd are biases. */
static int is_mfma_weight(const orc_net* m, int t) {
    /* W0 (t==0) is the gathered layer 1; the last weight (nt-2) is the head. */
    return (t % 2 == 0) && t != 0 && t != m->nt - 2;
}

static double* effective_weights(const orc_net* m, int t, int mode) {
    size_t R = (size_t)m->rows[t], C = (size_t)m->cols[t];
    double* w = (double*)malloc(R * C * sizeof(double));
    memcpy(w, m->T[t], R * C * sizeof(double));
    if (mode == 0 || t % 2 == 1) return w; /* biases stay float32 */
    if (mode == 1 || !is_mfma_weight(m, t)) {
        for (size_t i = 0; i < R * C; i++) w[i] = orc_bf16_round(w[i]);
        return w;
    }
    for (size_t n = 0; n < C; n++) {
        double mx = 0;
        for (size_t k = 0; k < R; k++) mx = fmax(mx, fabs(m->T[t][k * C + n]));
        float s = (float)(mx / 448.0); /* float32 quotient, correctly rounded */
        for (size_t k = 0; k < R; k++) {
            double q = 0.0;
            if (s > 0.0f) q = orc_e4m3_round((double)(float)(m->T[t][k * C + n] / (double)s));
            w[k * C + n] = q * (double)s;
        }
    }
    return w;
}

/* Per-column fp8 weight scales of MFMA tensor t (for tests). */
int orc_net_fp8_col_scales(const orc_net* m, int t, float* out) {
    size_t R = (size_t)m->rows[t], C = (size_t)m->cols[t];
    for (size_t n = 0; n < C; n++) {
        double mx = 0;
        for (size_t k = 0; k < R; k++) mx = fmax(mx, fabs(m->T[t][k * C + n]));
        out[n] = (float)(mx / 448.0);
    }
    return 1;
}

static double quant_act(double v, int mode, double scale) {
    if (mode == 1) return orc_bf16_round(v);
    if (mode == 2) return orc_e4m3_round(v / scale) * scale;
    return v;
}

/* ------------------------------------------------------------ forward */
/* Forward pass over n states (unpacked symbol bytes, P per state).
 * mode: 0 double, 1 bf16 operands, 2 fp8 operands (act_scale[n_act] needed).
 * y_out: n * n_out raw outputs.  act_max (nullable): per activation tensor,
 * the largest activation seen (used for calibration). */
int orc_net_forward(const orc_net* m, const uint8_t* states, int64_t n, int mode,
                    const double* act_scale, double* y_out, double* act_max) {
    double* W[MAXT];
    for (int t = 0; t < m->nt; t++) W[t] = effective_weights(m, t, mode);
    int maxw = m->n_in;
    for (int i = 0; i < m->n_dense; i++) if (m->dims[i] > maxw) maxw = m->dims[i];
    double* x = (double*)malloc((size_t)maxw * sizeof(double));
    double* t1 = (double*)malloc((size_t)maxw * sizeof(double));
    double* z = (double*)malloc((size_t)maxw * sizeof(double));
    int n_act = orc_net_n_act(m);
    if (act_max) for (int a = 0; a < n_act; a++) act_max[a] = 0.0;
    for (int64_t b = 0; b < n; b++) {
        const uint8_t* s = states + b * m->P;
        int act = 0, ti = 0;
        /* layer 1: gather-sum of one-hot rows */
        int H = m->dims[0];
        for (int j = 0; j < H; j++) z[j] = W[1][j];
        for (int p = 0; p < m->P; p++) {
            int row = p * m->S + s[p];
            for (int j = 0; j < H; j++) z[j] += W[0][(size_t)row * H + j];
        }
        for (int j = 0; j < H; j++) {
            double v = z[j] > 0 ? z[j] : 0.0;
            if (act_max && v > act_max[act]) act_max[act] = v;
            x[j] = quant_act(v, mode, act_scale ? act_scale[act] : 1.0);
        }
        act++;
        ti = 2;
        int K = H;
        /* dense layers */
        for (int i = 1; i < m->n_dense; i++) {
            int N = m->dims[i];
            for (int j = 0; j < N; j++) {
                double acc = 0.0;
                for (int k = 0; k < K; k++) acc += x[k] * W[ti][(size_t)k * N + j];
                z[j] = acc + W[ti + 1][j];
            }
            for (int j = 0; j < N; j++) {
                double v = z[j] > 0 ? z[j] : 0.0;
                if (act_max && v > act_max[act]) act_max[act] = v;
                x[j] = quant_act(v, mode, act_scale ? act_scale[act] : 1.0);
            }
            act++;
            ti += 2;
            K = N;
        }
        /* residual blocks */
        for (int r = 0; r < m->n_res; r++) {
            for (int j = 0; j < K; j++) {
                double acc = 0.0;
                for (int k = 0; k < K; k++) acc += x[k] * W[ti][(size_t)k * K + j];
                double v = acc + W[ti + 1][j];
                v = v > 0 ? v : 0.0;
                if (act_max && v > act_max[act]) act_max[act] = v;
                t1[j] = quant_act(v, mode, act_scale ? act_scale[act] : 1.0);
            }
            act++;
            for (int j = 0; j < K; j++) {
                double acc = 0.0;
                for (int k = 0; k < K; k++) acc += t1[k] * W[ti + 2][(size_t)k * K + j];
                double v = x[j] + acc + W[ti + 3][j];
                z[j] = v > 0 ? v : 0.0;
            }
            for (int j = 0; j < K; j++) {
                if (act_max && z[j] > act_max[act]) act_max[act] = z[j];
                x[j] = quant_act(z[j], mode, act_scale ? act_scale[act] : 1.0);
            }
            act++;
            ti += 4;
        }
        /* head */
        for (int o = 0; o < m->n_out; o++) {
            double acc = 0.0;
            for (int k = 0; k < K; k++) acc += x[k] * W[ti][(size_t)k * m->n_out + o];
            y_out[b * m->n_out + o] = acc + W[ti + 1][o];
        }
    }
    free(x); free(t1); free(z);
    for (int t = 0; t < m->nt; t++) free(W[t]);
    return 1;
}

/* ------------------------------------------------- one layer at a time
 * For layer-by-layer parity: the pre-activation z of one layer computed in
 * double precision from given (already quantised) inputs, together with
 * A = sum of |terms| (|x_k w_kn| over k, plus |bias| and |residual|), which
 * bounds the rounding error of any float32 evaluation order (the caller
 * applies ReLU and the storage rounding).  Activation index a as in the
 * forward pass: 0 = layer 1 (gathered from states), 1..n_dense-1 = dense
 * layers, then two per residual block (t, then x), n_act = the head.
 * x_in: n x K inputs (doubles, dequantised); r_in: n x N residual input for
 * the second layer of a residual block (else ignored, may be NULL).
 * Returns the output width, or 0 for a bad index. */
static int layer_tensor(const orc_net* m, int a) {
    /* each activation after layer 1, and the head, comes from one weight
       tensor, in file order */
    return 2 * a;
}

int orc_net_layer_width(const orc_net* m, int a) {
    if (a < 0 || a > orc_net_n_act(m)) return 0;
    return m->cols[layer_tensor(m, a)];
}

int orc_net_layer1(const orc_net* m, const uint8_t* states, int64_t n, int mode, double* z_out, double* abs_out) {
    double* W0 = effective_weights(m, 0, mode);
    int H = m->dims[0];
    for (int64_t b = 0; b < n; b++) {
        const uint8_t* s = states + b * m->P;
        double* z = z_out + b * H;
        double* A = abs_out + b * H;
        for (int j = 0; j < H; j++) { z[j] = m->T[1][j]; A[j] = fabs(m->T[1][j]); }
        for (int p = 0; p < m->P; p++) {
            const double* w = W0 + (size_t)(p * m->S + s[p]) * H;
            for (int j = 0; j < H; j++) { z[j] += w[j]; A[j] += fabs(w[j]); }
        }
    }
    free(W0);
    return H;
}

int orc_net_layer(const orc_net* m, int a, const double* x_in, const double* r_in, int64_t n, int mode,
                  double* z_out, double* abs_out) {
    int n_act = orc_net_n_act(m);
    if (a < 1 || a > n_act) return 0;
    int t = layer_tensor(m, a);
    int K = m->rows[t], N = m->cols[t];
    /* the second layer of residual block r produces activation n_dense + 2r + 1 */
    int residual = a < n_act && a >= m->n_dense && (a - m->n_dense) % 2 == 1;
    double* W = effective_weights(m, t, mode);
    for (int64_t b = 0; b < n; b++) {
        const double* x = x_in + b * K;
        for (int j = 0; j < N; j++) {
            double acc = 0.0, aa = 0.0;
            for (int k = 0; k < K; k++) {
                double term = x[k] * W[(size_t)k * N + j];
                acc += term;
                aa += fabs(term);
            }
            double bias = m->T[t + 1][j];
            acc += bias;
            aa += fabs(bias);
            if (residual) { acc += r_in[b * N + j]; aa += fabs(r_in[b * N + j]); }
            z_out[b * N + j] = acc;
            abs_out[b * N + j] = aa;
        }
    }
    free(W);
    return N;
}

/* Static fp8 activation scales: for each stored activation tensor, the
 * smallest power of two a with max|activation| / a <= 448 over a calibration
 * set, from the unquantised forward pass. */
int orc_net_calibrate(const orc_net* m, const uint8_t* states, int64_t n, double* scales) {
    int n_act = orc_net_n_act(m);
    double* mx = (double*)calloc((size_t)n_act, sizeof(double));
    double* tmp = (double*)malloc((size_t)n_act * sizeof(double));
    double* y = (double*)malloc((size_t)m->n_out * sizeof(double));
    for (int64_t b = 0; b < n; b++) {
        orc_net_forward(m, states + b * m->P, 1, 0, NULL, y, tmp);
        for (int a = 0; a < n_act; a++) if (tmp[a] > mx[a]) mx[a] = tmp[a];
    }
    for (int a = 0; a < n_act; a++) {
        if (!(mx[a] > 0)) { scales[a] = 1.0; continue; }
        int e = 0;
        while (448.0 * ldexp(1.0, e) < mx[a]) e++;
        while (448.0 * ldexp(1.0, e - 1) >= mx[a]) e--;
        scales[a] = ldexp(1.0, e);
    }
    free(mx); free(tmp); free(y);
    return n_act;
}

/* ------------------------------------------------------------ output rules */
/* mode 0 floor, 1 round-half-even, 2 real (floor reported). classic < 0: none. */
int orc_h_regression(double y, int mode, double offset, int classic) {
    if (!isfinite(y)) return classic >= 0 ? classic : 0;
    double v = y - offset;
    double r;
    if (mode == 1) {
        r = floor(v);
        double frac = v - r;
        if (frac > 0.5 || (frac == 0.5 && fmod(r, 2.0) != 0.0)) r += 1.0;
    } else {
        r = floor(v);
    }
    if (r < 0) r = 0;
    if (r > 1e9) r = 1e9;
    int h = (int)r;
    if (classic >= 0 && classic < h) h = classic;
    return h;
}

/* mode 3 quantile: smallest class whose cumulative softmax probability is at
 * least q (the last class if none); mode 4 arg-max (lowest index on ties).
 * Returns -1 when the output is undefined (a NaN or +infinite logit): the
 * caller falls back to the classic heuristic, or 0. */
int orc_h_classifier(const double* z, int n_out, int mode, double q) {
    for (int c = 0; c < n_out; c++) if (isnan(z[c]) || z[c] == INFINITY) return -1;
    if (mode == 4) {
        int best = 0;
        for (int c = 1; c < n_out; c++) if (z[c] > z[best]) best = c;
        return best;
    }
    double mx = z[0];
    for (int c = 1; c < n_out; c++) if (z[c] > mx) mx = z[c];
    double sum = 0.0;
    for (int c = 0; c < n_out; c++) sum += exp(z[c] - mx);
    double cdf = 0.0;
    for (int c = 0; c < n_out; c++) {
        cdf += exp(z[c] - mx) / sum;
        if (cdf >= q) return c;
    }
    return n_out - 1;
}

int orc_h_batch(const orc_net* m, const double* y, int64_t n, int mode, double q, double offset,
                const int32_t* classic, int32_t* h) {
    for (int64_t b = 0; b < n; b++) {
        if (m->head_kind == 1 || mode >= 3) {
            h[b] = orc_h_classifier(y + b * m->n_out, m->n_out, mode, q);
            if (h[b] < 0) h[b] = classic ? classic[b] : 0;
        }
        else
            h[b] = orc_h_regression(y[b * m->n_out], mode, offset, classic ? classic[b] : -1);
    }
    return 1;
}
