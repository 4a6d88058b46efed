/*
 * FP64 CPU oracle for the fused subdomain training step of domain-decomposed
 * PINN flow reconstruction (arXiv 2602.15883).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link or call
 * this file.  Only the test suite, the package's smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header, table or
 * constant with the HIP library; it is a plain, slow, per-point rendering of
 * the definitions, written so each line can be checked against the paper.
 *
 * What it computes (paper section 2.1 and 2.2):
 *   - the local expert: a fully connected tanh (or sin, section 3.2-3.3) MLP
 *     (x, t) -> (u, p)
 *     (section 2.1, network equation; section 2.2, "local expert"),
 *   - the derivatives the Navier-Stokes residuals need: d/dx_j, d/dt and
 *     d2/dx_j^2 of every output, carried through each layer in forward mode
 *     (the paper gets them from autograd; the values are the same),
 *   - the residuals r_1..r_d (momentum) and r_{d+1} (continuity)
 *     (section 2.1, residual definitions r1-r4),
 *   - the losses L_obs, L_PDE (section 2.1), L_gh_u, L_gh_p split in space and
 *     time parts (section 2.2, ghost consistency losses and the final local
 *     objective), plus an optional reference-anchor pressure term L_anc,
 *   - the exact gradient of the weighted loss with respect to every parameter
 *     (hand-derived adjoint of the forward above),
 *   - one Adam update (Algorithm 1, optimizer step), with the optional
 *     global-norm gradient clipping and step learning-rate decay of the 3D
 *     cylinder recipe (section 3.3, appendix B),
 *   - point queries: routing to the half-open subdomain box and (u, v, p, w)
 *     with vorticity w = v_x - u_y (section 3, stitching of local experts),
 *   - the ghost-target exchange with reference anchor normalisation
 *     (section 2.2, anchor-normalised pressure; Algorithm 1, exchange branch),
 *   - evaluation post-processing: stitched predictions, master anchor
 *     pinning, per-snapshot spatial-mean removal, relative L2 errors
 *     (section 3, relative L2 equation and pressure post-processing).
 *
 * Conventions (readings where the paper is silent):
 *   inputs xi = (x_1..x_d, t); outputs y = (u_1..u_d, p)
 *   parameters packed as W1[W][d_in], b1[W], W2[W][W], b2[W], ...,
 *   W_{H+1}[d_out][W], b_{H+1}[d_out]; row-major [out][in]
 *   channel c of a point: 0 = value, 1..d = d/dx_j, d+1 = d/dt,
 *   d+2..2d+1 = d2/dx_j^2  (C = 2d+2 channels)
 *   every MSE sums over components and divides by the number of points
 *   both ghost pressure parts divide by the subdomain's total ghost count
 *   masters use lambda_gh_p^space = 0 (section 2.2, asymmetric weighting)
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXC 8   /* 2*3 + 2 channels in 3D */

typedef struct {
  int dim, din, dout, W, H;
  int act;                 /* 0 = tanh, 1 = sin (the paper's cylinder networks) */
  const double *theta;
} net_t;

static int g_act = 0;      /* activation of the nets built by the entry points */

static void net_init(net_t *n, int dim, int W, int H, const double *theta) {
  n->dim = dim; n->din = dim + 1; n->dout = dim + 1; n->W = W; n->H = H;
  n->act = g_act;
  n->theta = theta;
}

/* activation sigma and its first three derivatives at z */
static void act_derivs(int act, double z, double *s, double *s1, double *s2, double *s3) {
  if (act == 1) {            /* sin: sin, cos, -sin, -cos */
    *s = sin(z); *s1 = cos(z); *s2 = -*s; *s3 = -*s1;
  } else {                   /* tanh: s, 1 - s^2, -2 s (1 - s^2), 2 (1 - s^2)(3 s^2 - 1) */
    *s = tanh(z); *s1 = 1.0 - *s * *s; *s2 = -2.0 * *s * *s1; *s3 = 2.0 * *s1 * (3.0 * *s * *s - 1.0);
  }
}

void or_set_activation(int act) { g_act = act; }

long or_nparams(int dim, int W, int H) {
  long din = dim + 1, dout = dim + 1;
  return W * din + W + (long)(H - 1) * (W * W + W) + dout * W + dout;
}

/* offsets of W_l and b_l inside the packed parameter vector, l = 1..H+1 */
static long off_w(const net_t *n, int l) {
  if (l == 1) return 0;
  long o = (long)n->W * n->din + n->W;
  o += (long)(l - 2) * ((long)n->W * n->W + n->W);
  return o;
}
static long off_b(const net_t *n, int l) {
  if (l == 1) return (long)n->W * n->din;
  if (l <= n->H) return off_w(n, l) + (long)n->W * n->W;
  return off_w(n, l) + (long)n->dout * n->W;
}

static int nch(int dim) { return 2 * dim + 2; }

/*
 * Forward pass of one point carrying C channels (C = 1: value only,
 * C = 2d+2: value, first and second derivatives).  Stores the pre-activation
 * z and the activation h of every hidden layer: z[l][c][k], h[l][c][k] for
 * l = 0..H-1 (layer l+1 of the paper's numbering), and the outputs y[c][o].
 */
static void forward_point(const net_t *n, const double *xi, int C,
                          double *z, double *h, double *y) {
  const int W = n->W, d = n->dim;
  const double *th = n->theta;
  for (int l = 0; l < n->H; l++) {
    double *zl = z + (long)l * C * W;
    double *hl = h + (long)l * C * W;
    if (l == 0) {
      /* input layer: z0 = W1 xi + b1; d z/d xi_j = W1[:, j]; second
       * derivatives of an affine map vanish */
      const double *W1 = th + off_w(n, 1), *b1 = th + off_b(n, 1);
      for (int k = 0; k < W; k++) {
        double s = b1[k];
        for (int j = 0; j < n->din; j++) s += W1[k * n->din + j] * xi[j];
        zl[k] = s;
        if (C > 1) {
          for (int j = 0; j <= d; j++) zl[(1 + j) * W + k] = W1[k * n->din + j];
          for (int j = 0; j < d; j++) zl[(d + 2 + j) * W + k] = 0.0;
        }
      }
    } else {
      const double *Wl = th + off_w(n, l + 1), *bl = th + off_b(n, l + 1);
      const double *hp = h + (long)(l - 1) * C * W;
      for (int c = 0; c < C; c++)
        for (int k = 0; k < W; k++) {
          double s = (c == 0) ? bl[k] : 0.0;
          for (int i = 0; i < W; i++) s += Wl[k * W + i] * hp[c * W + i];
          zl[c * W + k] = s;
        }
    }
    /* activation with the chain rule: h = sigma(z0); h_j = sigma'(z0) z_j;
     * h_jj = sigma''(z0) z_j^2 + sigma'(z0) z_jj */
    for (int k = 0; k < W; k++) {
      double s, s1, s2, s3;
      act_derivs(n->act, zl[k], &s, &s1, &s2, &s3);
      hl[k] = s;
      if (C > 1) {
        for (int j = 0; j <= d; j++) hl[(1 + j) * W + k] = s1 * zl[(1 + j) * W + k];
        for (int j = 0; j < d; j++) {
          double zj = zl[(1 + j) * W + k];
          hl[(d + 2 + j) * W + k] = s2 * zj * zj + s1 * zl[(d + 2 + j) * W + k];
        }
      }
    }
  }
  /* linear output layer */
  const int L = n->H + 1;
  const double *Wo = th + off_w(n, L), *bo = th + off_b(n, L);
  const double *hH = h + (long)(n->H - 1) * C * W;
  for (int c = 0; c < C; c++)
    for (int o = 0; o < n->dout; o++) {
      double s = (c == 0) ? bo[o] : 0.0;
      for (int k = 0; k < W; k++) s += Wo[o * W + k] * hH[c * W + k];
      y[c * n->dout + o] = s;
    }
}

/*
 * Adjoint of forward_point: given ybar[c][o] = dL/dy^c_o for this point,
 * add dL/dtheta into grad.  z, h are the stored forward values.
 */
static void backward_point(const net_t *n, const double *xi, int C,
                           const double *z, const double *h, const double *ybar,
                           double *grad, double *hbar, double *zbar) {
  const int W = n->W, d = n->dim, L = n->H + 1;
  const double *th = n->theta;
  /* output layer: dW_out += ybar^c (h_H^c)^T, db_out += ybar^0,
   * hbar_H^c = W_out^T ybar^c */
  {
    const double *Wo = th + off_w(n, L);
    double *gW = grad + off_w(n, L), *gb = grad + off_b(n, L);
    const double *hH = h + (long)(n->H - 1) * C * W;
    for (int c = 0; c < C; c++)
      for (int o = 0; o < n->dout; o++) {
        double yb = ybar[c * n->dout + o];
        if (yb == 0.0) continue;
        for (int k = 0; k < W; k++) gW[o * W + k] += yb * hH[c * W + k];
        if (c == 0) gb[o] += yb;
      }
    for (int c = 0; c < C; c++)
      for (int k = 0; k < W; k++) {
        double s = 0.0;
        for (int o = 0; o < n->dout; o++) s += Wo[o * W + k] * ybar[c * n->dout + o];
        hbar[c * W + k] = s;
      }
  }
  for (int l = n->H - 1; l >= 0; l--) {
    const double *zl = z + (long)l * C * W;
    /* activation adjoint (reverse of the chain rule above) */
    for (int k = 0; k < W; k++) {
      double s, s1, s2, s3;
      act_derivs(n->act, zl[k], &s, &s1, &s2, &s3);
      double z0bar = s1 * hbar[k];
      if (C > 1) {
        for (int j = 0; j <= d; j++) {
          /* h_j = s1 z_j: d/dz_j -> s1, d/dz0 -> s2 z_j */
          double zj = zl[(1 + j) * W + k], hb = hbar[(1 + j) * W + k];
          zbar[(1 + j) * W + k] = s1 * hb;
          z0bar += s2 * zj * hb;
        }
        for (int j = 0; j < d; j++) {
          /* h_jj = s2 z_j^2 + s1 z_jj */
          double zj = zl[(1 + j) * W + k], zjj = zl[(d + 2 + j) * W + k];
          double hb = hbar[(d + 2 + j) * W + k];
          zbar[(d + 2 + j) * W + k] = s1 * hb;
          zbar[(1 + j) * W + k] += 2.0 * s2 * zj * hb;
          z0bar += (s3 * zj * zj + s2 * zjj) * hb;
        }
      }
      zbar[k] = z0bar;
    }
    if (l > 0) {
      /* hidden layer l+1: dW += zbar^c (h_l^c)^T, db += zbar^0,
       * hbar_{l}^c = W^T zbar^c */
      const double *Wl = th + off_w(n, l + 1);
      double *gW = grad + off_w(n, l + 1), *gb = grad + off_b(n, l + 1);
      const double *hp = h + (long)(l - 1) * C * W;
      for (int c = 0; c < C; c++)
        for (int k = 0; k < W; k++) {
          double zb = zbar[c * W + k];
          if (zb == 0.0) continue;
          for (int i = 0; i < W; i++) gW[k * W + i] += zb * hp[c * W + i];
          if (c == 0) gb[k] += zb;
        }
      for (int c = 0; c < C; c++)
        for (int i = 0; i < W; i++) {
          double s = 0.0;
          for (int k = 0; k < W; k++) s += Wl[k * W + i] * zbar[c * W + k];
          hbar[c * W + i] = s;
        }
    } else {
      /* input layer: z0 = W1 xi + b1, z_j = W1[:, j] */
      double *gW = grad + off_w(n, 1), *gb = grad + off_b(n, 1);
      for (int k = 0; k < W; k++) {
        for (int j = 0; j < n->din; j++) {
          double g = zbar[k] * xi[j];
          if (C > 1) g += zbar[(1 + j) * W + k];
          gW[k * n->din + j] += g;
        }
        gb[k] += zbar[k];
      }
    }
  }
}

/* ---------------------------------------------------------------------- */
/* Residuals: section 2.1, incompressible Navier-Stokes, r1..r4.          */
/* y[c][o] holds the channel stack of one point.                           */
/* ---------------------------------------------------------------------- */
static void residual_point(int d, double nu, const double *y, double *r) {
  const int D = d + 1;
#define Y(c, o) y[(c) * D + (o)]
  for (int i = 0; i < d; i++) {
    double conv = 0.0, lap = 0.0;
    for (int j = 0; j < d; j++) {
      conv += Y(0, j) * Y(1 + j, i);     /* u_j d_j u_i */
      lap += Y(d + 2 + j, i);            /* d_jj u_i */
    }
    r[i] = Y(1 + d, i) + conv + Y(1 + i, d) - nu * lap;
  }
  double div = 0.0;
  for (int j = 0; j < d; j++) div += Y(1 + j, j);
  r[d] = div;
#undef Y
}

/*
 * Seeds dL/dy for a PDE point, with rb[k] = 2 lambda_PDE r_k / N_pde
 * (derivative of lambda_PDE/N_pde * sum_k r_k^2 with respect to each channel).
 */
static void pde_seed(int d, double nu, const double *y, const double *rb, double *yb) {
  const int D = d + 1, C = nch(d);
#define Y(c, o) y[(c) * D + (o)]
#define YB(c, o) yb[(c) * D + (o)]
  for (int i = 0; i < C * D; i++) yb[i] = 0.0;
  for (int i = 0; i < d; i++) {
    /* r_k contains u_j d_j u_k: d/du_i -> d_i u_k */
    double s = 0.0;
    for (int k = 0; k < d; k++) s += rb[k] * Y(1 + i, k);
    YB(0, i) = s;
    for (int j = 0; j < d; j++) {
      YB(1 + j, i) = rb[i] * Y(0, j) + (i == j ? rb[d] : 0.0);
      YB(d + 2 + j, i) = -nu * rb[i];
    }
    YB(1 + d, i) = rb[i];
  }
  for (int j = 0; j < d; j++) YB(1 + j, d) = rb[j];   /* d_j p in r_j */
#undef Y
#undef YB
}

/* ---------------------------------------------------------------------- */
/* Public entry points (all arrays are plain double, row-major)           */
/* ---------------------------------------------------------------------- */

static int set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
  return omp_get_max_threads();
#else
  (void)nthreads;
  return 1;
#endif
}

int or_threads(int nthreads) { return set_threads(nthreads); }

/* All channels y[n][C][d_out] of the network at points x[n][d_in]. */
void or_channels(int dim, int W, int H, const double *theta,
                 const double *x, long n, double *y) {
  net_t nt; net_init(&nt, dim, W, H, theta);
  const int C = nch(dim);
#pragma omp parallel
  {
    double *z = malloc(sizeof(double) * (size_t)H * C * W);
    double *h = malloc(sizeof(double) * (size_t)H * C * W);
#pragma omp for schedule(static)
    for (long p = 0; p < n; p++)
      forward_point(&nt, x + p * nt.din, C, z, h, y + p * C * nt.dout);
    free(z); free(h);
  }
}

/* Value outputs y[n][d_out] only. */
void or_values(int dim, int W, int H, const double *theta,
               const double *x, long n, double *y) {
  net_t nt; net_init(&nt, dim, W, H, theta);
#pragma omp parallel
  {
    double *z = malloc(sizeof(double) * (size_t)H * W);
    double *h = malloc(sizeof(double) * (size_t)H * W);
#pragma omp for schedule(static)
    for (long p = 0; p < n; p++)
      forward_point(&nt, x + p * nt.din, 1, z, h, y + p * nt.dout);
    free(z); free(h);
  }
}

/* Residuals r[n][d+1] from channel stacks y[n][C][d_out]. */
void or_residuals(int dim, double nu, const double *y, long n, double *r) {
  const int C = nch(dim), D = dim + 1;
  for (long p = 0; p < n; p++) residual_point(dim, nu, y + p * C * D, r + p * D);
}

/*
 * Loss and gradient of one subdomain.
 *   lam[6] = {obs, pde, gh_u, gh_p_space, gh_p_time, anc}
 *   loss[7] = {L_obs, L_PDE, L_gh_u, L_gh_p^space, L_gh_p^time, L_anc, L}
 *     (terms unweighted, total weighted; lambda_gh_p^space taken as 0 when
 *      is_master, section 2.2 asymmetric weighting)
 *   grad[P] (may be NULL): dL/dtheta
 *   gh_kind[i]: 0 = spatial interface, 1 = temporal interface
 *   Points are processed in static blocks by thread; each thread sums into
 *   its own accumulator and the accumulators are added in thread order.
 */
/* weights of the velocity components in L_obs and L_gh_u (section 3.3 uses
 * (1, 5, 100) for (u, v, w)); all ones by default */
static double g_cw[3] = {1.0, 1.0, 1.0};
void or_set_component_weights(const double *w) {
  for (int i = 0; i < 3; i++) g_cw[i] = w ? w[i] : 1.0;
}

void or_loss_grad(int dim, int W, int H, double nu, const double *lam, int is_master,
                  const double *theta,
                  const double *pde_x, long n_pde,
                  const double *obs_x, const double *obs_u, long n_obs,
                  const double *gh_x, const double *gh_up, const unsigned char *gh_kind, long n_gh,
                  const double *anc_x, const double *anc_p, long n_anc,
                  double *loss, double *grad) {
  net_t nt; net_init(&nt, dim, W, H, theta);
  const int C = nch(dim), D = dim + 1, d = dim;
  const long P = or_nparams(dim, W, H);
  const double l_obs = lam[0], l_pde = lam[1], l_ghu = lam[2];
  const double l_sp = is_master ? 0.0 : lam[3], l_tm = lam[4], l_anc = lam[5];
  int nthr = set_threads(0);
  double *tl = calloc((size_t)nthr * 6, sizeof(double));
  double *tg = grad ? calloc((size_t)nthr * P, sizeof(double)) : NULL;

#pragma omp parallel
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    double *z = malloc(sizeof(double) * (size_t)H * C * W);
    double *h = malloc(sizeof(double) * (size_t)H * C * W);
    double *hb = malloc(sizeof(double) * (size_t)C * W);
    double *zb = malloc(sizeof(double) * (size_t)C * W);
    double y[OR_MAXC * 4], yb[OR_MAXC * 4], r[4], rb[4];
    double *myl = tl + tid * 6;
    double *myg = tg ? tg + (size_t)tid * P : NULL;

    /* collocation points: L_PDE = (1/N) sum_n sum_k r_k^2 */
#pragma omp for schedule(static)
    for (long p = 0; p < n_pde; p++) {
      const double *xi = pde_x + p * D;
      forward_point(&nt, xi, C, z, h, y);
      residual_point(d, nu, y, r);
      double s = 0.0;
      for (int k = 0; k < D; k++) { s += r[k] * r[k]; rb[k] = 2.0 * l_pde * r[k] / (double)n_pde; }
      myl[1] += s;
      if (myg) {
        pde_seed(d, nu, y, rb, yb);
        backward_point(&nt, xi, C, z, h, yb, myg, hb, zb);
      }
    }
    /* observation points: L_obs = (1/N) sum_n ||u - u_obs||^2 */
#pragma omp for schedule(static)
    for (long p = 0; p < n_obs; p++) {
      const double *xi = obs_x + p * D;
      forward_point(&nt, xi, 1, z, h, y);
      double s = 0.0;
      for (int o = 0; o < D; o++) yb[o] = 0.0;
      for (int i = 0; i < d; i++) {
        double e = y[i] - obs_u[p * d + i];
        s += g_cw[i] * e * e;
        yb[i] = 2.0 * l_obs * g_cw[i] * e / (double)n_obs;
      }
      myl[0] += s;
      if (myg) backward_point(&nt, xi, 1, z, h, yb, myg, hb, zb);
    }
    /* ghost points: L_gh_u and L_gh_p^{space|time}, each over N_gh */
#pragma omp for schedule(static)
    for (long p = 0; p < n_gh; p++) {
      const double *xi = gh_x + p * D;
      const double *tgt = gh_up + p * D;
      forward_point(&nt, xi, 1, z, h, y);
      double s = 0.0;
      for (int i = 0; i < d; i++) {
        double e = y[i] - tgt[i];
        s += g_cw[i] * e * e;
        yb[i] = 2.0 * l_ghu * g_cw[i] * e / (double)n_gh;
      }
      myl[2] += s;
      double ep = y[d] - tgt[d];
      int temporal = gh_kind[p] != 0;
      myl[temporal ? 4 : 3] += ep * ep;
      yb[d] = 2.0 * (temporal ? l_tm : l_sp) * ep / (double)n_gh;
      if (myg) backward_point(&nt, xi, 1, z, h, yb, myg, hb, zb);
    }
    /* anchor points: L_anc = (1/N_anc) sum (p - p_a)^2 */
#pragma omp for schedule(static)
    for (long p = 0; p < n_anc; p++) {
      const double *xi = anc_x + p * D;
      forward_point(&nt, xi, 1, z, h, y);
      double ep = y[d] - anc_p[p];
      myl[5] += ep * ep;
      for (int o = 0; o < D; o++) yb[o] = 0.0;
      yb[d] = 2.0 * l_anc * ep / (double)n_anc;
      if (myg) backward_point(&nt, xi, 1, z, h, yb, myg, hb, zb);
    }
    free(z); free(h); free(hb); free(zb);
  }

  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int t = 0; t < nthr; t++)
    for (int k = 0; k < 6; k++) acc[k] += tl[t * 6 + k];
  loss[0] = n_obs ? acc[0] / (double)n_obs : 0.0;
  loss[1] = n_pde ? acc[1] / (double)n_pde : 0.0;
  loss[2] = n_gh ? acc[2] / (double)n_gh : 0.0;
  loss[3] = n_gh ? acc[3] / (double)n_gh : 0.0;
  loss[4] = n_gh ? acc[4] / (double)n_gh : 0.0;
  loss[5] = n_anc ? acc[5] / (double)n_anc : 0.0;
  loss[6] = l_obs * loss[0] + l_pde * loss[1] + l_ghu * loss[2] +
            l_sp * loss[3] + l_tm * loss[4] + l_anc * loss[5];
  if (grad) {
    for (long i = 0; i < P; i++) {
      double s = 0.0;
      for (int t = 0; t < nthr; t++) s += tg[(size_t)t * P + i];
      grad[i] = s;
    }
  }
  free(tl); free(tg);
}

/* Gradient clipping by global norm (section 3.3: maximum norm 1.0):
 * g <- g * min(1, c / ||g||_2).  Returns ||g||_2 before clipping. */
double or_clip_grad(double *g, long P, double c) {
  double ss = 0.0;
  for (long i = 0; i < P; i++) ss += g[i] * g[i];
  double nrm = sqrt(ss);
  if (c > 0.0 && nrm > c) {
    double f = c / nrm;
    for (long i = 0; i < P; i++) g[i] *= f;
  }
  return nrm;
}

/* Step decay of the learning rate (appendix B, "LR factor & interval"):
 * lr_t = lr * factor^floor((t - 1) / interval); interval <= 0 keeps lr. */
double or_step_lr(double lr, double factor, long interval, long t) {
  if (interval <= 0) return lr;
  return lr * pow(factor, (double)((t - 1) / interval));
}

/* Adam with bias correction, step t >= 1 (Algorithm 1 optimizer step). */
void or_adam(double *theta, double *m, double *v, const double *g, long P, long t,
             double lr, double b1, double b2, double eps) {
  double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
  for (long i = 0; i < P; i++) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    double mh = m[i] / c1, vh = v[i] / c2;
    theta[i] -= lr * mh / (sqrt(vh) + eps);
  }
}

/*
 * Routing (section 3, stitching): the subdomain whose half-open box
 * [lo, hi) contains the point; a coordinate equal to the global upper
 * bound (the largest hi over all boxes on that axis) counts as inside.
 * boxes[s][2][d_in] = {lo, hi}.  Returns -1 for points in no box.
 */
void or_route(int dim, int n_sub, const double *boxes, const double *x, long n, int *sub) {
  const int D = dim + 1;
  double gmax[4];
  for (int a = 0; a < D; a++) {
    gmax[a] = -INFINITY;
    for (int s = 0; s < n_sub; s++)
      if (boxes[(s * 2 + 1) * D + a] > gmax[a]) gmax[a] = boxes[(s * 2 + 1) * D + a];
  }
  for (long p = 0; p < n; p++) {
    int found = -1;
    for (int s = 0; s < n_sub && found < 0; s++) {
      int in = 1;
      for (int a = 0; a < D; a++) {
        double lo = boxes[(s * 2) * D + a], hi = boxes[(s * 2 + 1) * D + a];
        double c = x[p * D + a];
        int ok = (c >= lo) && (c < hi || (c == hi && hi == gmax[a]));
        if (!ok) { in = 0; break; }
      }
      if (in) found = s;
    }
    sub[p] = found;
  }
}

/*
 * Query of 2D networks: out[n][4] = (u, v, p, v_x - u_y) of the subdomain
 * each point routes to; thetas[s] points at subdomain s's parameters.
 * Points that route nowhere get NaN.
 */
void or_query2d(int W, int H, int n_sub, const double *const *thetas,
                const double *boxes, const double *x, long n, double *out) {
  const int dim = 2, D = 3, C = nch(dim);
  int *sub = malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  or_route(dim, n_sub, boxes, x, n, sub);
#pragma omp parallel
  {
    double *z = malloc(sizeof(double) * (size_t)H * C * W);
    double *h = malloc(sizeof(double) * (size_t)H * C * W);
    double y[OR_MAXC * 4];
#pragma omp for schedule(static)
    for (long p = 0; p < n; p++) {
      if (sub[p] < 0) { for (int k = 0; k < 4; k++) out[p * 4 + k] = NAN; continue; }
      net_t nt; net_init(&nt, dim, W, H, thetas[sub[p]]);
      forward_point(&nt, x + p * D, C, z, h, y);
      out[p * 4 + 0] = y[0];
      out[p * 4 + 1] = y[1];
      out[p * 4 + 2] = y[2];
      out[p * 4 + 3] = y[1 * D + 1] - y[2 * D + 0];  /* v_x - u_y */
    }
    free(z); free(h);
  }
  free(sub);
}

/*
 * Ghost-target exchange (section 2.2 anchor normalisation, Algorithm 1
 * exchange branch).  For ghost points x[n][d_in] of a receiving subdomain,
 * whose owner is the neighbour with parameters theta_nb:
 *   u_nbr = u_nb(x), p_nbr = p_nb(x) - [nb is master] p_nb(x_anc, t(x)).
 * out[n][d_out].
 */
void or_exchange(int dim, int W, int H, const double *theta_nb, int nb_is_master,
                 const double *x_anc, const double *x, long n, double *out) {
  net_t nt; net_init(&nt, dim, W, H, theta_nb);
  const int D = dim + 1;
#pragma omp parallel
  {
    double *z = malloc(sizeof(double) * (size_t)H * W);
    double *h = malloc(sizeof(double) * (size_t)H * W);
    double y[4], ya[4], xa[4];
#pragma omp for schedule(static)
    for (long p = 0; p < n; p++) {
      forward_point(&nt, x + p * D, 1, z, h, y);
      for (int o = 0; o < D; o++) out[p * D + o] = y[o];
      if (nb_is_master) {
        for (int a = 0; a < dim; a++) xa[a] = x_anc[a];
        xa[dim] = x[p * D + dim];          /* the ghost point's own time */
        forward_point(&nt, xa, 1, z, h, ya);
        out[p * D + dim] = y[dim] - ya[dim];
      }
    }
    free(z); free(h);
  }
}

/*
 * Evaluation post-processing (section 3, relative L2 error equation and the
 * pressure post-processing that follows it).  Points x[n][d_in] are grouped
 * in snapshots: snapshot k holds points snap_off[k] .. snap_off[k+1]-1.
 *   1. predictions of the subdomain each point routes to (stitching),
 *   2. points in master subdomains: p~ = p - p(x_anc, t) with the same network,
 *   3. per snapshot, the spatial mean of p~ and of the reference p is removed,
 *   4. err[i] = ||u_i,pred - u_i,ref|| / ||u_i,ref|| (i < d),
 *      err[d] = the same over all velocity components together,
 *      err[d+1] = the same for the processed pressure.
 * ref[n][d_in] = (u_1..u_d, p).  thetas[s], is_master[s] per subdomain.
 */
void or_evaluate(int dim, int W, int H, int n_sub, const double *const *thetas,
                 const int *is_master, const double *boxes, const double *x_anc,
                 const double *x, long n, const double *ref, const long *snap_off, int n_snap,
                 double *err) {
  const int D = dim + 1;
  int *sub = malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  double *pred = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * D);
  or_route(dim, n_sub, boxes, x, n, sub);
#pragma omp parallel
  {
    double *z = malloc(sizeof(double) * (size_t)H * W);
    double *h = malloc(sizeof(double) * (size_t)H * W);
    double y[4], ya[4], xa[4];
#pragma omp for schedule(static)
    for (long p = 0; p < n; p++) {
      if (sub[p] < 0) { for (int o = 0; o < D; o++) pred[p * D + o] = NAN; continue; }
      net_t nt; net_init(&nt, dim, W, H, thetas[sub[p]]);
      forward_point(&nt, x + p * D, 1, z, h, y);
      for (int o = 0; o < D; o++) pred[p * D + o] = y[o];
      if (is_master[sub[p]]) {
        for (int a = 0; a < dim; a++) xa[a] = x_anc[a];
        xa[dim] = x[p * D + dim];
        forward_point(&nt, xa, 1, z, h, ya);
        pred[p * D + dim] -= ya[dim];
      }
    }
    free(z); free(h);
  }
  double num[4] = {0, 0, 0, 0}, den[4] = {0, 0, 0, 0}, nump = 0.0, denp = 0.0;
  for (int k = 0; k < n_snap; k++) {
    long a = snap_off[k], b = snap_off[k + 1];
    double mp = 0.0, mr = 0.0;
    for (long p = a; p < b; p++) { mp += pred[p * D + dim]; mr += ref[p * D + dim]; }
    if (b > a) { mp /= (double)(b - a); mr /= (double)(b - a); }
    for (long p = a; p < b; p++) {
      for (int i = 0; i < dim; i++) {
        double e = pred[p * D + i] - ref[p * D + i];
        num[i] += e * e;
        den[i] += ref[p * D + i] * ref[p * D + i];
      }
      double ep = (pred[p * D + dim] - mp) - (ref[p * D + dim] - mr);
      double rp = ref[p * D + dim] - mr;
      nump += ep * ep;
      denp += rp * rp;
    }
  }
  double nv = 0.0, dv = 0.0;
  for (int i = 0; i < dim; i++) {
    err[i] = sqrt(num[i] / den[i]);
    nv += num[i];
    dv += den[i];
  }
  err[dim] = sqrt(nv / dv);
  err[dim + 1] = sqrt(nump / denp);
  free(sub); free(pred);
}
