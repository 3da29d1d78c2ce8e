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
 *   loss = mean over samples and interior points of (y_4(p, 0) - target)^2,
 *          or the cut-level objective of orc_net_judge_loss_grad.
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

/* index-sum parity of grid point q */
static int parity(const Geo *g, int q)
{
    int G = g->G;
    return (q % G + (q / G) % G + q / (G * G)) & 1;
}

/* sum over the 2 dim axis neighbours of q of a[nb] (0 outside the interior) */
static double axis_sum(const Geo *g, const double *a, int q)
{
    int st[3] = {1, g->G, g->G * g->G};
    double s = 0;
    for (int ax = 0; ax < g->dim; ax++)
        for (int sg = -1; sg <= 1; sg += 2) {
            int nb = q + sg * st[ax];
            if (interior(g, nb)) s += a[nb];
        }
    return s;
}

static void backward(const Geo *g, int B, const double *act, const double *w, double *dY, double *grad);

/* loss (mean squared error over samples and interior points) and its
 * gradient with respect to w (same layout); returns NaN on bad arguments */
double orc_net_loss_grad(int dim, int B, const double *in, const double *target, const double *w,
                         double *grad)
{
    Geo g;
    if (geo(dim, &g) || B < 1) return NAN;
    size_t per = (size_t)B * g.pts * C;
    double *act = forward(&g, B, in, w);
    double *dY = (double *)calloc(per, sizeof(double));
    if (!act || !dY) { free(act); free(dY); return NAN; }
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
    backward(&g, B, act, w, dY, grad);
    free(act);
    free(dY);
    return loss;
}

/* The objective the coarse kernel judges the network by: the network output
 * y, taken at the points of the cut level that it shares with the level
 * below (index sum even), goes through that level's own red-black Jacobi
 * step for Lap v = x with the residual weighted by pj (its over-relaxation
 * parameter; x the network input, all in the network's units, spacing 1):
 * first the odd points v = (sum of the 2 dim neighbours' y - pj x) / (2 dim),
 * then the even ones from the new odd values; the loss is the mean over
 * samples and interior points of rho^2, rho = x - (sum of neighbours' v - 2 dim
 * v), i.e. the squared reduction of the cut level's residual norm when x is
 * normalised to unit rms.  Gradient by the chain rule through the step (a
 * linear map) and the network. */
double orc_net_judge_loss_grad(int dim, int B, const double *in, const double *w, double pj, double *grad)
{
    Geo g;
    if (geo(dim, &g) || B < 1) return NAN;
    size_t per = (size_t)B * g.pts * C;
    double *act = forward(&g, B, in, w);
    double *dY = (double *)calloc(per, sizeof(double));
    double *y = (double *)calloc((size_t)g.pts, sizeof(double));
    double *v = (double *)calloc((size_t)g.pts, sizeof(double));
    double *rho = (double *)calloc((size_t)g.pts, sizeof(double));
    double *dv = (double *)calloc((size_t)g.pts, sizeof(double));
    double *dvf = (double *)calloc((size_t)g.pts, sizeof(double));
    if (!act || !dY || !y || !v || !rho || !dv || !dvf) {
        free(act); free(dY); free(y); free(v); free(rho); free(dv); free(dvf);
        return NAN;
    }
    int G2 = g.G - 2;
    double cnt = (double)B * G2 * G2 * (dim == 3 ? G2 : 1), d2 = 2.0 * dim;
    double loss = 0;
    for (int b = 0; b < B; b++) {
        const double *x = in + (size_t)b * g.pts;
        for (int q = 0; q < g.pts; q++) {
            y[q] = (interior(&g, q) && !parity(&g, q)) ? act[per * NL + ((size_t)b * g.pts + q) * C] : 0.0;
            v[q] = rho[q] = dv[q] = dvf[q] = 0.0;
        }
        for (int q = 0; q < g.pts; q++)   /* odd points from the network's even values */
            if (interior(&g, q) && parity(&g, q)) v[q] = (axis_sum(&g, y, q) - pj * x[q]) / d2;
        for (int q = 0; q < g.pts; q++)   /* even points from the new odd values */
            if (interior(&g, q) && !parity(&g, q)) v[q] = (axis_sum(&g, v, q) - pj * x[q]) / d2;
        for (int q = 0; q < g.pts; q++)
            if (interior(&g, q)) {
                rho[q] = x[q] - (axis_sum(&g, v, q) - d2 * v[q]);
                loss += rho[q] * rho[q];
            }
        /* d loss / d v = -L (2 rho / cnt): L is symmetric with the zero boundary */
        for (int q = 0; q < g.pts; q++)
            if (interior(&g, q)) dv[q] = -(axis_sum(&g, rho, q) - d2 * rho[q]) * 2.0 / cnt;
        /* through the even half-step: each odd point feeds its even neighbours */
        for (int q = 0; q < g.pts; q++) {
            if (!interior(&g, q) || !parity(&g, q)) continue;
            double s = 0;
            int st[3] = {1, g.G, g.G * g.G};
            for (int ax = 0; ax < dim; ax++)
                for (int sg = -1; sg <= 1; sg += 2) {
                    int nb = q + sg * st[ax];
                    if (interior(&g, nb)) s += dv[nb];
                }
            dvf[q] = dv[q] + s / d2;
        }
        /* through the odd half-step onto the network's even outputs */
        for (int q = 0; q < g.pts; q++)
            if (interior(&g, q) && !parity(&g, q)) dY[((size_t)b * g.pts + q) * C] = axis_sum(&g, dvf, q) / d2;
    }
    loss /= cnt;
    backward(&g, B, act, w, dY, grad);
    free(act); free(dY); free(y); free(v); free(rho); free(dv); free(dvf);
    return loss;
}

/* gradient of the loss with respect to w from the gradient dY with respect
 * to the last layer's output (channel 0); dY is overwritten */
static void backward(const Geo *gp, int B, const double *act, const double *w, double *dY, double *grad)
{
    const Geo g = *gp;
    const int dim = g.dim;
    (void)dim;
    size_t per = (size_t)B * g.pts * C;
    size_t WL = (size_t)g.T * C * C;
    double *dX = (double *)calloc(per, sizeof(double));
    if (!dX) { for (size_t i = 0; i < NL * WL; i++) grad[i] = NAN; return; }
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
    free(dX);
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
