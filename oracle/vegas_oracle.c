/*
 * vegas_oracle.c — plain FP64 CPU oracle for one Vegas iteration.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may include, link,
 * load or call this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark do. It shares no code, header, table or constant with
 * the HIP implementation.
 *
 * What it follows. The paper (VegasFlow, arXiv:2010.09341) names the method
 * without stating it: Monte Carlo integration by importance sampling on an
 * adaptive grid, the Vegas algorithm of Lepage (Sec. 1), driven iteration by
 * iteration so that each iteration's sampling informs the grid of the next
 * (Sec. 3.2), with a user integrand that maps a batch of points in the unit
 * hypercube to one value per point and several iterations per run (the code
 * example of Sec. 3.1). The steps below spell out that method in the order
 * an iteration takes them:
 *
 *   O1 grid        uniform edges e[d][i] = i/nb
 *   O2 draw        Philox4x32-10 words, counter (n_lo, n_hi, t, d/4), key = seed
 *   O3 map         word -> (bin k, fraction) -> x_d, Jacobian factor nb*Delta
 *   O4 weight      w = f(x) * prod_d nb*Delta_d
 *   O5 moments     S1 = sum w, S2 = sum w^2 (compensated), I = S1/N,
 *                  sigma^2 = (S2/N - I^2)/(N-1), clamped at 0
 *   O6 histogram   h[d][k_d] += w^2 for every dimension d (compensated)
 *   O7 refine      smooth, normalise, compress with exponent alpha,
 *                  redistribute edges so every new bin holds equal mass
 *   O8 combine     inverse-variance average over iterations, chi^2/dof
 *
 * Where the paper is silent the readings are: the RNG family and its counter
 * layout; the integer bin index k = floor(r*nb/2^32) with the fraction taken
 * at the centre of the remaining 2^-32 cell; the w^2 histogram; the
 * (1,1,1)/3 smoothing with (1,1)/2 at the ends; r_i = ((1-p_i)/(-ln p_i))^alpha;
 * the unbiased per-iteration variance; inverse-variance combination including
 * the first iteration; non-finite weights counted and contributing zero.
 *
 * Precision: every floating-point step is IEEE binary64, compiled without
 * fast-math and without FMA contraction.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define VO_OK 0
#define VO_EINVAL (-1)

#define VO_F_CONST 0
#define VO_F_SUM 1
#define VO_F_GAUSS 2
#define VO_F_LO_TOY 3
#define VO_F_RAMBO24 4
#define VO_F_BW_FLAT 5

/* ---------------------------------------------------------------------------
 * O2: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
 * as easy as 1, 2, 3", SC'11). A round multiplies counter words 0 and 2 by
 * two fixed odd constants to 64-bit products, and builds the next counter
 * from the high halves xor-ed with the other two words and the round key,
 * and from the low halves. The key is bumped by two Weyl constants between
 * rounds. Ten rounds.
 * ------------------------------------------------------------------------- */
void vo_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                      uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u; /* golden ratio Weyl increment */
      k1 += 0xBB67AE85u; /* sqrt(3)-1 Weyl increment */
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* The 32-bit random word that drives dimension d of event n in iteration t. */
static void vo_event_words(uint64_t seed, uint32_t t, uint64_t n, int dim,
                           uint32_t *words) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int j = 0; 4 * j < dim; ++j) {
    uint32_t ctr[4] = {(uint32_t)n, (uint32_t)(n >> 32), t, (uint32_t)j};
    uint32_t out[4];
    vo_philox4x32_10(ctr, key, out);
    for (int i = 0; i < 4 && 4 * j + i < dim; ++i) words[4 * j + i] = out[i];
  }
}

/* ---------------------------------------------------------------------------
 * O1: the starting grid is uniform.
 * ------------------------------------------------------------------------- */
int vo_uniform_grid(int dim, int nb, double *edges) {
  if (dim < 1 || nb < 2 || !edges) return VO_EINVAL;
  for (int d = 0; d < dim; ++d)
    for (int i = 0; i <= nb; ++i) edges[d * (nb + 1) + i] = (double)i / nb;
  return VO_OK;
}

/* ---------------------------------------------------------------------------
 * O3: one dimension of the grid map. The word r is read as the point
 * y = r/2^32 of [0,1); y*nb splits into the bin index k (integer part, exact)
 * and the position inside the bin. The position is the centre of the 2^-32
 * cell that r selects, so it never touches the bin edges. The point is
 * x = e_k + frac * (e_{k+1} - e_k); the map's Jacobian in this dimension is
 * nb * (e_{k+1} - e_k).
 * ------------------------------------------------------------------------- */
void vo_map_dim(int nb, const double *e, uint32_t r, double *x, int *k,
                double *jac_factor) {
  uint64_t prod = (uint64_t)r * (uint64_t)nb;
  int bin = (int)(prod >> 32);
  uint32_t rem = (uint32_t)prod;
  double frac = ((double)rem + 0.5) / 4294967296.0;
  double width = e[bin + 1] - e[bin];
  *x = e[bin] + frac * width;
  *k = bin;
  *jac_factor = (double)nb * width;
}

/* ---------------------------------------------------------------------------
 * RAMBO (Kleiss, Stirling, Ellis, Comput. Phys. Commun. 40 (1986) 359), named
 * among the standard Monte Carlo tools in Sec. 2: flat massless n-body phase
 * space from 4n uniforms. Four isotropic massless momenta with energies drawn
 * from q0 e^{-q0} are generated, then one Lorentz boost and one scaling take
 * their sum to (sqrt_s, 0, 0, 0). The phase-space weight is constant:
 * (pi/2)^(n-1) s^(n-2) / ((n-1)! (n-2)!), with no (2 pi) factors.
 * p is [4][4] as (E, px, py, pz).
 * ------------------------------------------------------------------------- */
double vo_rambo4(double sqrt_s, const double *u, double *p) {
  const double pi = 3.14159265358979323846;
  double q[4][4];
  double Q[4] = {0, 0, 0, 0};
  for (int i = 0; i < 4; ++i) {
    double cth = 2.0 * u[4 * i + 0] - 1.0;
    double sth = sqrt(1.0 - cth * cth);
    double phi = 2.0 * pi * u[4 * i + 1];
    double e = -log(u[4 * i + 2] * u[4 * i + 3]);
    q[i][0] = e;
    q[i][1] = e * sth * cos(phi);
    q[i][2] = e * sth * sin(phi);
    q[i][3] = e * cth;
    for (int m = 0; m < 4; ++m) Q[m] += q[i][m];
  }
  double M = sqrt(Q[0] * Q[0] - Q[1] * Q[1] - Q[2] * Q[2] - Q[3] * Q[3]);
  double b[3] = {-Q[1] / M, -Q[2] / M, -Q[3] / M};
  double gamma = Q[0] / M;
  double a = 1.0 / (1.0 + gamma);
  double scale = sqrt_s / M;
  for (int i = 0; i < 4; ++i) {
    double bq = b[0] * q[i][1] + b[1] * q[i][2] + b[2] * q[i][3];
    p[4 * i + 0] = scale * (gamma * q[i][0] + bq);
    for (int m = 0; m < 3; ++m)
      p[4 * i + 1 + m] = scale * (q[i][1 + m] + b[m] * q[i][0] + a * bq * b[m]);
  }
  double s = sqrt_s * sqrt_s;
  /* (pi/2)^3 s^2 / (3! 2!) */
  return (pi / 2.0) * (pi / 2.0) * (pi / 2.0) * s * s / (6.0 * 2.0);
}

/* ---------------------------------------------------------------------------
 * O4: the integrands. par/np are the caller's raw parameters; defaults apply
 * when np is 0. Every function is written in its plain product/quotient form.
 *   CONST    f = 1
 *   SUM      f = sum_d x_d            (the toy of the Sec. 3.1 code example)
 *   GAUSS    f = prod_d exp(-(x_d-c_d)^2/a^2) / (a sqrt(pi));
 *            par = {a, c_0..c_{D-1}} (centres default to 0.5)
 *   LO_TOY   x = (x1, x2, u_cos, u_phi); s_hat = x1 x2 s;
 *            f = g(x1) g(x2) (1+c^2) BW(s_hat)/s_hat * 2 * 2 pi,
 *            c = 2 u_cos - 1, g(x) = x^-1/2 (1-x)^3,
 *            BW(s_hat) = (m G/pi) / ((s_hat-m^2)^2 + m^2 G^2),
 *            zero unless sqrt(s_hat) > cut;
 *            par = {sqrt_s, m, G, cut} = {13000, 91.19, 2.5, 20}
 *   RAMBO24  16 uniforms -> 4 massless momenta (RAMBO) at sqrt_s;
 *            mode 0: f = W * prod over cyclic neighbours (01)(12)(23)(30) of
 *            1/s_ij, zero if any of those s_ij <= cut_frac * s;
 *            mode 1: f = W (the phase-space volume);
 *            par = {sqrt_s, cut_frac, mode} = {1000, 0.01, 0}
 *   BW_FLAT  f = (G/(2 pi)) / ((x_0-m)^2 + G^2/4), flat in the other
 *            dimensions; par = {m, G} = {0.5, 0.02}
 * ------------------------------------------------------------------------- */
static double vo_par(const double *par, int np, int i, double dflt) {
  return (par && i < np) ? par[i] : dflt;
}

int vo_integrand_check(int id, int dim, int np) {
  if (np < 0) return VO_EINVAL;
  switch (id) {
    case VO_F_CONST:
    case VO_F_SUM:
      return VO_OK;
    case VO_F_GAUSS:
      return (np == 0 || np == 1 || np == 1 + dim) ? VO_OK : VO_EINVAL;
    case VO_F_LO_TOY:
      return (dim == 4 && np <= 4) ? VO_OK : VO_EINVAL;
    case VO_F_RAMBO24:
      return (dim == 16 && np <= 3) ? VO_OK : VO_EINVAL;
    case VO_F_BW_FLAT:
      return np <= 2 ? VO_OK : VO_EINVAL;
    default:
      return VO_EINVAL;
  }
}

double vo_integrand(int id, int dim, const double *par, int np,
                    const double *x) {
  const double pi = 3.14159265358979323846;
  switch (id) {
    case VO_F_CONST:
      return 1.0;
    case VO_F_SUM: {
      double s = 0.0;
      for (int d = 0; d < dim; ++d) s += x[d];
      return s;
    }
    case VO_F_GAUSS: {
      double a = vo_par(par, np, 0, 0.1);
      double f = 1.0;
      for (int d = 0; d < dim; ++d) {
        double c = (np == 1 + dim) ? par[1 + d] : 0.5;
        double z = x[d] - c;
        f *= exp(-(z * z) / (a * a)) / (a * sqrt(pi));
      }
      return f;
    }
    case VO_F_LO_TOY: {
      double sqrt_s = vo_par(par, np, 0, 13000.0);
      double m = vo_par(par, np, 1, 91.19);
      double G = vo_par(par, np, 2, 2.5);
      double cut = vo_par(par, np, 3, 20.0);
      double x1 = x[0], x2 = x[1];
      double c = 2.0 * x[2] - 1.0;
      double s_hat = x1 * x2 * (sqrt_s * sqrt_s);
      if (!(sqrt(s_hat) > cut)) return 0.0;
      double g1 = pow(x1, -0.5) * pow(1.0 - x1, 3.0);
      double g2 = pow(x2, -0.5) * pow(1.0 - x2, 3.0);
      double dm = s_hat - m * m;
      double bw = (m * G / pi) / (dm * dm + m * m * G * G);
      return g1 * g2 * (1.0 + c * c) * bw / s_hat * 2.0 * (2.0 * pi);
    }
    case VO_F_RAMBO24: {
      double sqrt_s = vo_par(par, np, 0, 1000.0);
      double cut_frac = vo_par(par, np, 1, 0.01);
      int mode = (int)vo_par(par, np, 2, 0.0);
      double p[16];
      double W = vo_rambo4(sqrt_s, x, p);
      if (mode == 1) return W;
      double s = sqrt_s * sqrt_s;
      double f = W;
      for (int i = 0; i < 4; ++i) {
        int j = (i + 1) % 4;
        double dot = p[4 * i] * p[4 * j] - p[4 * i + 1] * p[4 * j + 1] -
                     p[4 * i + 2] * p[4 * j + 2] - p[4 * i + 3] * p[4 * j + 3];
        double sij = 2.0 * dot;
        if (!(sij > cut_frac * s)) return 0.0;
        f /= sij;
      }
      return f;
    }
    case VO_F_BW_FLAT: {
      double m = vo_par(par, np, 0, 0.5);
      double G = vo_par(par, np, 1, 0.02);
      double z = x[0] - m;
      return (G / (2.0 * pi)) / (z * z + G * G / 4.0);
    }
    default:
      return NAN;
  }
}

/* ---------------------------------------------------------------------------
 * Neumaier's compensated summation (Neumaier 1974): keeps the rounding error
 * of every addition in a second accumulator. Sums are taken in event order.
 * ------------------------------------------------------------------------- */
typedef struct {
  double s, c;
} vo_sum;

static void vo_sum_add(vo_sum *a, double v) {
  double t = a->s + v;
  if (fabs(a->s) >= fabs(v))
    a->c += (a->s - t) + v;
  else
    a->c += (v - t) + a->s;
  a->s = t;
}

static double vo_sum_value(const vo_sum *a) { return a->s + a->c; }

static int vo_check_grid(int dim, int nb) {
  return (dim >= 1 && dim <= 64 && nb >= 2 && nb <= 4096) ? VO_OK : VO_EINVAL;
}

/* O2-O4 for one event: its point, bins, Jacobian and weight. */
static double vo_event(int dim, int nb, const double *edges, int id,
                       const double *par, int np, uint64_t seed, uint32_t t,
                       uint64_t n, double *x, int *k) {
  uint32_t words[64];
  vo_event_words(seed, t, n, dim, words);
  double jac = 1.0;
  for (int d = 0; d < dim; ++d) {
    double jf;
    vo_map_dim(nb, edges + (size_t)d * (nb + 1), words[d], &x[d], &k[d], &jf);
    jac *= jf;
  }
  return vo_integrand(id, dim, par, np, x) * jac;
}

/* Per-event weights of events first .. first+count-1 (test hook). */
int vo_weights(int dim, int nb, const double *edges, int id, const double *par,
               int np, uint64_t seed, uint32_t t, uint64_t first, int64_t count,
               double *w_out) {
  if (vo_check_grid(dim, nb) || vo_integrand_check(id, dim, np) || count < 0)
    return VO_EINVAL;
  double x[64];
  int k[64];
  for (int64_t i = 0; i < count; ++i)
    w_out[i] = vo_event(dim, nb, edges, id, par, np, seed, t, first + i, x, k);
  return VO_OK;
}

/* Points and bin indices of events first .. first+count-1 (test hook). */
int vo_points(int dim, int nb, const double *edges, uint64_t seed, uint32_t t,
              uint64_t first, int64_t count, double *x_out, int *k_out,
              double *jac_out) {
  if (vo_check_grid(dim, nb) || count < 0) return VO_EINVAL;
  uint32_t words[64];
  for (int64_t i = 0; i < count; ++i) {
    vo_event_words(seed, t, first + i, dim, words);
    double jac = 1.0;
    for (int d = 0; d < dim; ++d) {
      double jf;
      vo_map_dim(nb, edges + (size_t)d * (nb + 1), words[d],
                 &x_out[i * dim + d], &k_out[i * dim + d], &jf);
      jac *= jf;
    }
    jac_out[i] = jac;
  }
  return VO_OK;
}

/* ---------------------------------------------------------------------------
 * One iteration, O2-O6. hist_out is [dim][nb]. Events whose weight is not
 * finite are counted in *n_nonfinite and contribute nothing.
 * ------------------------------------------------------------------------- */
int vo_iterate(int dim, int nb, const double *edges, int id, const double *par,
               int np, int64_t n_events, uint64_t seed, uint32_t t, double *I,
               double *sigma, double *hist_out, int64_t *n_nonfinite) {
  if (vo_check_grid(dim, nb) || vo_integrand_check(id, dim, np) || n_events < 2)
    return VO_EINVAL;
  vo_sum s1 = {0, 0}, s2 = {0, 0};
  vo_sum *h = (vo_sum *)calloc((size_t)dim * nb, sizeof(vo_sum));
  if (!h) return VO_EINVAL;
  int64_t bad = 0;
  double x[64];
  int k[64];
  for (int64_t n = 0; n < n_events; ++n) {
    double w = vo_event(dim, nb, edges, id, par, np, seed, t, (uint64_t)n, x, k);
    if (!isfinite(w)) {
      ++bad;
      continue;
    }
    double w2 = w * w;
    vo_sum_add(&s1, w);
    vo_sum_add(&s2, w2);
    for (int d = 0; d < dim; ++d) vo_sum_add(&h[(size_t)d * nb + k[d]], w2);
  }
  double N = (double)n_events;
  double mean = vo_sum_value(&s1) / N;
  double var = (vo_sum_value(&s2) / N - mean * mean) / (N - 1.0);
  *I = mean;
  *sigma = sqrt(var > 0.0 ? var : 0.0);
  if (hist_out)
    for (size_t i = 0; i < (size_t)dim * nb; ++i) hist_out[i] = vo_sum_value(&h[i]);
  if (n_nonfinite) *n_nonfinite = bad;
  free(h);
  return VO_OK;
}

/* ---------------------------------------------------------------------------
 * O7: grid refinement, dimension by dimension.
 *  1. smooth the histogram: mean of the bin and its neighbours,
 *     (h0+h1)/2 and (h_{nb-2}+h_{nb-1})/2 at the ends;
 *  2. normalise to p_i = s_i / sum s; a dimension with sum 0 is left as is;
 *  3. compress: r_i = ((1-p_i)/(-ln p_i))^alpha, r_i = 0 for p_i = 0 and
 *     r_i = 1 for p_i = 1;
 *  4. running sums C_0 = 0, C_{i+1} = C_i + r_i, left to right; delta = C_nb/nb;
 *  5. new edge j (0 < j < nb) lies in the old bin k with C_k < j delta <=
 *     C_{k+1}, at the fraction (j delta - C_k)/r_k of its width;
 *  6. the outer edges stay 0 and 1.
 * ------------------------------------------------------------------------- */
int vo_refine(int dim, int nb, const double *edges, const double *hist,
              double alpha, double *new_edges) {
  if (vo_check_grid(dim, nb) || !(alpha >= 0.0)) return VO_EINVAL;
  double *s = (double *)malloc(sizeof(double) * nb);
  double *r = (double *)malloc(sizeof(double) * nb);
  double *C = (double *)malloc(sizeof(double) * (nb + 1));
  double *ne = (double *)malloc(sizeof(double) * (nb + 1));
  if (!s || !r || !C || !ne) {
    free(s); free(r); free(C); free(ne);
    return VO_EINVAL;
  }
  for (int d = 0; d < dim; ++d) {
    const double *h = hist + (size_t)d * nb;
    const double *e = edges + (size_t)d * (nb + 1);
    double *out = new_edges + (size_t)d * (nb + 1);
    s[0] = (h[0] + h[1]) / 2.0;
    for (int i = 1; i < nb - 1; ++i) s[i] = (h[i - 1] + h[i] + h[i + 1]) / 3.0;
    s[nb - 1] = (h[nb - 2] + h[nb - 1]) / 2.0;
    double S = 0.0;
    for (int i = 0; i < nb; ++i) S += s[i];
    if (!(S > 0.0)) {
      for (int i = 0; i <= nb; ++i) out[i] = e[i];
      continue;
    }
    for (int i = 0; i < nb; ++i) {
      double p = s[i] / S;
      if (p <= 0.0)
        r[i] = 0.0;
      else if (p >= 1.0)
        r[i] = 1.0;
      else
        r[i] = pow((1.0 - p) / (-log(p)), alpha);
    }
    C[0] = 0.0;
    for (int i = 0; i < nb; ++i) C[i + 1] = C[i] + r[i];
    double delta = C[nb] / nb;
    ne[0] = 0.0;
    int k = 0;
    for (int j = 1; j < nb; ++j) {
      double target = j * delta;
      while (k < nb - 1 && !(C[k + 1] >= target)) ++k;
      ne[j] = e[k] + (target - C[k]) / r[k] * (e[k + 1] - e[k]);
    }
    ne[nb] = 1.0;
    for (int i = 0; i <= nb; ++i) out[i] = ne[i];
  }
  free(s); free(r); free(C); free(ne);
  return VO_OK;
}

/* ---------------------------------------------------------------------------
 * O8: combine iterations by inverse-variance weighting; chi^2 per degree of
 * freedom of the iteration results about the combined mean. An iteration with
 * sigma_t = 0 makes the combination that iteration's value with sigma 0.
 * ------------------------------------------------------------------------- */
int vo_combine(int n, const double *I_t, const double *sigma_t, double *I,
               double *sigma, double *chi2_dof) {
  if (n < 1) return VO_EINVAL;
  for (int t = 0; t < n; ++t)
    if (!(sigma_t[t] > 0.0)) {
      *I = I_t[t];
      *sigma = 0.0;
      *chi2_dof = 0.0;
      return VO_OK;
    }
  double sw = 0.0, swi = 0.0;
  for (int t = 0; t < n; ++t) {
    double wt = 1.0 / (sigma_t[t] * sigma_t[t]);
    sw += wt;
    swi += wt * I_t[t];
  }
  double mean = swi / sw;
  double chi2 = 0.0;
  for (int t = 0; t < n; ++t) {
    double z = (I_t[t] - mean) / sigma_t[t];
    chi2 += z * z;
  }
  *I = mean;
  *sigma = 1.0 / sqrt(sw);
  *chi2_dof = n > 1 ? chi2 / (n - 1) : 0.0;
  return VO_OK;
}

/* A whole run: n_iter iterations from the uniform grid, refining after every
 * iteration but the last. Per-iteration results go to I_t/sigma_t; the final
 * grid to edges_out (may be NULL). */
int vo_run(int dim, int nb, int id, const double *par, int np, int64_t n_events,
           uint64_t seed, int n_iter, double alpha, double *I_t,
           double *sigma_t, double *edges_out, int64_t *n_nonfinite) {
  if (vo_check_grid(dim, nb) || n_iter < 1) return VO_EINVAL;
  size_t ne = (size_t)dim * (nb + 1);
  double *e = (double *)malloc(sizeof(double) * ne);
  double *e2 = (double *)malloc(sizeof(double) * ne);
  double *h = (double *)malloc(sizeof(double) * (size_t)dim * nb);
  if (!e || !e2 || !h) {
    free(e); free(e2); free(h);
    return VO_EINVAL;
  }
  vo_uniform_grid(dim, nb, e);
  int64_t bad_total = 0;
  int rc = VO_OK;
  for (int t = 0; t < n_iter && rc == VO_OK; ++t) {
    int64_t bad = 0;
    rc = vo_iterate(dim, nb, e, id, par, np, n_events, seed, (uint32_t)t,
                    &I_t[t], &sigma_t[t], h, &bad);
    bad_total += bad;
    if (rc == VO_OK && t + 1 < n_iter) {
      rc = vo_refine(dim, nb, e, h, alpha, e2);
      memcpy(e, e2, sizeof(double) * ne);
    }
  }
  if (edges_out) memcpy(edges_out, e, sizeof(double) * ne);
  if (n_nonfinite) *n_nonfinite = bad_total;
  free(e); free(e2); free(h);
  return rc;
}
