/*
 * CPU oracle of the learned coarse correction: a network of four 3x3 (2D) or
 * 3x3x3 (3D) convolutions with 16 channels (1 -> 16 -> 16 -> 16 -> 1), ReLU
 * after the first three, no bias, zero padding outside the interior of the
 * grid (the Dirichlet boundary); mean-squared-error loss, its gradient by the
 * chain rule, and an Adam step.
 *
 * TEST INFRASTRUCTURE ONLY: plain double-precision loops written from the
 * definition of a convolution; the GPU library never links it.  Tests run it
 * on the GPU's bf16-rounded weights and inputs.
 *
 * Conventions (shared by definition with the GPU path, not by code):
 *   grid   [B][G][G] (2D, G = 17) or [B][G][G][G] (3D, G = 9), natural
 *          order, x fastest, interior 1..G-2, boundary 0;
 *   weight [layer 4][tap T][cin 16][cout 16], T = 3^dim, tap index
 *          (dy+1)*3 + (dx+1) in 2D, ((dz+1)*3 + (dy+1))*3 + (dx+1) in 3D;
 *          layer 0 reads only cin 0, layer 3 writes only cout 0;
 *   y_{l+1}(p, co) = sum_t sum_ci y_l(p + off(t), ci) w[l][t][ci][co] at
 *          interior p, then ReLU for l < 3; y_0 = input in channel 0;
 *   loss = mean over samples and interior points of (y_4(p, 0) - target)^2.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define C 16
#define NL 4

typedef struct {
    int dim, G, T, pts;     /* pts = G^dim points per sample */
    int off[27];            /* linear offset of each tap */
} Geo;

static int geo(int dim, Geo *g)
{
    if (dim != 2 && dim != 3) return -1;
    g->dim = dim;
    g->G = dim == 2 ? 17 : 9;
    g->T = dim == 2 ? 9 : 27;
    g->pts = dim == 2 ? g->G * g->G : g->G * g->G * g->G;
    for (int t = 0; t < g->T; t++) {
        int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
        g->off[t] = dx + g->G * dy + (dim == 3 ? g->G * g->G * dz : 0);
    }
    return 0;
}

static int interior(const Geo *g, int q)
{
    int G = g->G;
    int x = q % G, y = (q / G) % G, z = q / (G * G);
    if (x < 1 || x > G - 2 || y < 1 || y > G - 2) return 0;
    if (g->dim == 3 && (z < 1 || z > G - 2)) return 0;
    return 1;
}

/* all activations: act[l][b][q][c], l = 0..NL */
static double *forward(const Geo *g, int B, const double *in, const double *w)
{
    size_t per = (size_t)B * g->pts * C;
    size_t WL = (size_t)g->T * C * C;
    double *a = (double *)calloc(per * (NL + 1) + 1, sizeof(double));
    if (!a) return NULL;
    for (int b = 0; b < B; b++)
        for (int q = 0; q < g->pts; q++)
            if (interior(g, q)) a[((size_t)b * g->pts + q) * C] = in[(size_t)b * g->pts + q];
    for (int l = 0; l < NL; l++) {
        const double *X = a + per * l;
        double *Y = a + per * (l + 1);
        const double *W = w + WL * l;
        for (int b = 0; b < B; b++)
            for (int q = 0; q < g->pts; q++) {
                if (!interior(g, q)) continue;
                for (int co = 0; co < C; co++) {
                    double s = 0;
                    for (int t = 0; t < g->T; t++) {
                        const double *x = X + ((size_t)b * g->pts + q + g->off[t]) * C;
                        for (int ci = 0; ci < C; ci++) s += x[ci] * W[((size_t)t * C + ci) * C + co];
                    }
                    if (l < NL - 1 && s < 0) s = 0;
                    Y[((size_t)b * g->pts + q) * C + co] = s;
                }
            }
    }
    return a;
}

/* out: [B][pts], channel 0 of the last layer (0 on the boundary); 0 or -1 */
int orc_net_forward(int dim, int B, const double *in, const double *w, double *out)
{
    Geo g;
    if (geo(dim, &g) || B < 0) return -1;
    double *a = forward(&g, B, in, w);
    if (!a) return -1;
    size_t per = (size_t)B * g.pts * C;
    for (size_t q = 0; q < (size_t)B * g.pts; q++) out[q] = a[per * NL + q * C];
    free(a);
    return 0;
}

/* loss (mean squared error over samples and interior points) and its
 * gradient with respect to w (same layout); returns NaN on bad arguments */
double orc_net_loss_grad(int dim, int B, const double *in, const double *target, const double *w,
                         double *grad)
{
    Geo g;
    if (geo(dim, &g) || B < 1) return NAN;
    size_t per = (size_t)B * g.pts * C;
    size_t WL = (size_t)g.T * C * C;
    double *act = forward(&g, B, in, w);
    double *dY = (double *)calloc(per, sizeof(double));
    double *dX = (double *)calloc(per, sizeof(double));
    if (!act || !dY || !dX) { free(act); free(dY); free(dX); return NAN; }
    int G2 = g.G - 2;
    double cnt = (double)B * G2 * G2 * (dim == 3 ? G2 : 1);
    double loss = 0;
    for (int b = 0; b < B; b++)
        for (int q = 0; q < g.pts; q++) {
            if (!interior(&g, q)) continue;
            size_t s = (size_t)b * g.pts + q;
            double e = act[per * NL + s * C] - target[s];
            loss += e * e;
            dY[s * C] = 2 * e / cnt;
        }
    loss /= cnt;
    memset(grad, 0, sizeof(double) * NL * WL);
    for (int l = NL - 1; l >= 0; l--) {
        /* dY: gradient with respect to the output of layer l (masked) */
        const double *X = act + per * l;
        const double *W = w + WL * l;
        double *gW = grad + WL * l;
        for (int b = 0; b < B; b++)
            for (int q = 0; q < g.pts; q++) {
                if (!interior(&g, q)) continue;
                const double *dy = dY + ((size_t)b * g.pts + q) * C;
                for (int t = 0; t < g.T; t++) {
                    const double *x = X + ((size_t)b * g.pts + q + g.off[t]) * C;
                    for (int ci = 0; ci < C; ci++)
                        for (int co = 0; co < C; co++) gW[((size_t)t * C + ci) * C + co] += x[ci] * dy[co];
                }
            }
        if (l == 0) break;
        memset(dX, 0, per * sizeof(double));
        for (int b = 0; b < B; b++)
            for (int q = 0; q < g.pts; q++) {
                if (!interior(&g, q)) continue;
                const double *dy = dY + ((size_t)b * g.pts + q) * C;
                for (int t = 0; t < g.T; t++) {
                    int src = q + g.off[t];
                    if (!interior(&g, src)) continue;   /* padding is not an activation */
                    double *dx = dX + ((size_t)b * g.pts + src) * C;
                    for (int ci = 0; ci < C; ci++) {
                        double s = 0;
                        for (int co = 0; co < C; co++) s += dy[co] * W[((size_t)t * C + ci) * C + co];
                        dx[ci] += s;
                    }
                }
            }
        /* through the ReLU that produced X (layer l-1's output) */
        for (size_t q = 0; q < per; q++) dY[q] = X[q] > 0 ? dX[q] : 0;
    }
    /* the padded channels of the first and last layer are not parameters */
    for (int t = 0; t < g.T; t++)
        for (int ci = 0; ci < C; ci++)
            for (int co = 0; co < C; co++) {
                if (ci != 0) grad[((size_t)t * C + ci) * C + co] = 0;
                if (co != 0) grad[WL * 3 + ((size_t)t * C + ci) * C + co] = 0;
            }
    free(act);
    free(dY);
    free(dX);
    return loss;
}

/* One Adam step (Kingma and Ba, Algorithm 1) on n parameters, bias-corrected
 * with the step number t >= 1: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * w -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps). */
void orc_net_adam(int n, double *w, double *m, double *v, const double *g, int t, double lr, double b1,
                  double b2, double eps)
{
    double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
    for (int i = 0; i < n; i++) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        w[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}
