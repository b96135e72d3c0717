/*
 * FP64 CPU oracle for the all-pairs GEMPE coding cost and its gradient.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library path may call this file; only the
 * tests, the smoke check and the benchmark's CPU-baseline leg load it.  It shares no
 * source, header, table or constant with the GPU library.
 *
 * What it computes (Sec. II-B of the paper, "Predictive Entropy PE"):
 *   s+(delta) = 1/2 - 1/2 erf((delta - mu)/(sqrt2 sigma))   edge probability
 *   s-(delta) = 1/2 + 1/2 erf((delta - mu)/(sqrt2 sigma))   non-edge probability
 *   dl+/- = -log2 s+/-                                        description length, bits
 *   dl(i,j) = dl+(|x_i - x_j|) if (i,j) in E, dl- otherwise
 *   DL = sum_{i<j} dl(i,j);  PE = DL / N  (Eq. 2 at fixed mu, sigma; N = n(n-1)/2)
 * and the gradient of DL with respect to every coordinate:
 *   g_i = sum_{j != i} (d dl(i,j)/d delta) (x_i - x_j) / delta_ij,
 * with the contribution of a coincident pair (delta = 0) taken as 0, the same
 * convention the weighted-majorization update uses for s_ij (Eq. 5).
 *
 * Evaluation of s+/- uses 1/2 -+ 1/2 erf(z) = 1/2 erfc(+-z), which is the same number
 * without the cancellation of the printed form; below tau = -35 (where erfc of the
 * argument approaches the double underflow) the standard asymptotic series of the
 * normal tail is used (Abramowitz and Stegun 26.2.12).  Loops are plain brute force:
 * every row i runs over every j != i (each unordered pair is evaluated from both
 * sides), edge membership comes from marking row i's CSR neighbours in a dense flag
 * array.  OpenMP splits rows over threads; the loss is summed over rows in fixed order.
 *
 * Weighted majorization (Sec. II-C, Eqs. 3-5): the parabola weight w_ij is half the
 * second derivative of dl at the current distance (matching first and second
 * derivatives), d_ij follows from matching the first derivative, and Eq. 5 gives the
 * new coordinates.  The printed Eq. 3 carries 2/(pi ln 2) in its first term where the
 * second derivative gives 1/(pi ln 2); this oracle follows the derivative-matching
 * requirement that the paper states, not the printed coefficient.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_LN2 0.69314718055994530941723212145818
#define ORACLE_SQRT2 1.41421356237309504880168872420970
#define ORACLE_LOG_SQRT_2PI 0.91893853320467274178032973640562 /* log(sqrt(2 pi)) */

/* Mills-ratio series factor S(t) = 1 - t^-2 + 3 t^-4 - 15 t^-6 + 105 t^-8 - 945 t^-10,
 * with Phi(t) ~ phi(t) S(t) / |t| as t -> -infinity (A&S 26.2.12). */
static double tail_series(double t) {
    double q = 1.0 / (t * t);
    return 1.0 + q * (-1.0 + q * (3.0 + q * (-15.0 + q * (105.0 + q * (-945.0)))));
}

/* log Phi(t) for the standard normal CDF Phi. */
static double log_Phi(double t) {
    if (t < -35.0) {
        return -0.5 * t * t - log(-t) - ORACLE_LOG_SQRT_2PI + log(tail_series(t));
    }
    if (t < 0.0) {
        return log(0.5 * erfc(-t / ORACLE_SQRT2));
    }
    return log1p(-0.5 * erfc(t / ORACLE_SQRT2));
}

/* phi(t) / Phi(t). */
static double mills_inv(double t) {
    if (t < -35.0) {
        return -t / tail_series(t);
    }
    double phi = exp(-0.5 * t * t - ORACLE_LOG_SQRT_2PI);
    double Phi = (t < 0.0) ? 0.5 * erfc(-t / ORACLE_SQRT2) : 1.0 - 0.5 * erfc(t / ORACLE_SQRT2);
    return phi / Phi;
}

/*
 * One vertex pair at distance delta.
 *   dl  : description length in bits, dl+ for an edge, dl- otherwise
 *   d1  : d dl / d delta
 *   d2  : d^2 dl / d delta^2
 * With tau = a (delta - mu)/sigma, a = -1 for an edge and +1 for a non-edge,
 * s = Phi(tau), so dl = -log2 Phi(tau), d1 = -(a/sigma) R / ln2 and
 * d2 = (tau R + R^2) / (sigma^2 ln 2), where R = phi(tau)/Phi(tau).
 */
void oracle_pair(double delta, int is_edge, double mu, double sigma,
                 double *dl, double *d1, double *d2) {
    double a = is_edge ? -1.0 : 1.0;
    double tau = a * (delta - mu) / sigma;
    double R = mills_inv(tau);
    if (dl) *dl = -log_Phi(tau) / ORACLE_LN2;
    if (d1) *d1 = -(a / sigma) * R / ORACLE_LN2;
    if (d2) *d2 = (tau * R + R * R) / (sigma * sigma * ORACLE_LN2);
}

/* Marks the CSR neighbours of row i in flag[] (1), returns nothing. */
static void mark_row(const int64_t *row_ptr, const int32_t *col_idx, int i, unsigned char *flag,
                     unsigned char value) {
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) flag[col_idx[e]] = value;
}

/*
 * Per-row brute force for a list of rows.
 *   rows      : the rows to evaluate (nrows of them); NULL means all rows 0..n-1
 *   X         : n x d, row-major, float64
 *   grad      : nrows x d output (row r of grad belongs to rows[r]); may be NULL
 *   row_loss  : nrows output, L_i = sum_{j != i} dl(i, j); may be NULL
 *   upper_loss: nrows output, U_i = sum_{j > i} dl(i, j); may be NULL
 *   upper_hits: nrows output, number of edges (i, j) with j > i recognised; may be NULL
 *   zsum      : nrows output, z_i = sum_{j != i} w_ij (Eq. 5 denominator); may be NULL
 *   ysum      : nrows x d output, y_i = sum_{j != i} w_ij (x_j + s_ij (x_i - x_j)); may be NULL
 *   abs_slope : nrows output, A_i = sum_{j != i} |d dl(i,j) / d delta| (the scale of the terms
 *               that cancel in g_i; used for gradient tolerances); may be NULL
 */
void oracle_rows(int n, int d, const double *X, const int64_t *row_ptr, const int32_t *col_idx,
                 double mu, double sigma, int nrows, const int64_t *rows, double *grad,
                 double *row_loss, double *upper_loss, int64_t *upper_hits, double *zsum,
                 double *ysum, double *abs_slope) {
    if (rows == NULL) nrows = n;
#pragma omp parallel
    {
        unsigned char *flag = (unsigned char *)calloc((size_t)n, 1);
        double *gi = (double *)malloc(sizeof(double) * (size_t)d);
        double *yi = (double *)malloc(sizeof(double) * (size_t)d);
#pragma omp for schedule(dynamic, 1)
        for (int r = 0; r < nrows; ++r) {
            int i = rows ? (int)rows[r] : r;
            const double *xi = X + (size_t)i * d;
            mark_row(row_ptr, col_idx, i, flag, 1);
            double L = 0.0, U = 0.0, z = 0.0, A = 0.0;
            int64_t hits = 0;
            for (int k = 0; k < d; ++k) gi[k] = 0.0, yi[k] = 0.0;
            for (int j = 0; j < n; ++j) {
                if (j == i) continue;
                const double *xj = X + (size_t)j * d;
                double r2 = 0.0;
                for (int k = 0; k < d; ++k) {
                    double t = xi[k] - xj[k];
                    r2 += t * t;
                }
                double delta = sqrt(r2);
                int edge = flag[j] != 0;
                double dl, d1, d2;
                oracle_pair(delta, edge, mu, sigma, &dl, &d1, &d2);
                L += dl;
                A += fabs(d1);
                if (j > i) {
                    U += dl;
                    hits += edge;
                }
                double c = (delta > 0.0) ? d1 / delta : 0.0;
                for (int k = 0; k < d; ++k) gi[k] += c * (xi[k] - xj[k]);
                if (zsum || ysum) {
                    /* parabola fit at the current distance: w = dl''/2, d = delta - dl'/(2w) */
                    double w = 0.5 * d2;
                    double dij = delta - d1 / (2.0 * w);
                    double s = (delta > 0.0) ? dij / delta : 0.0;
                    z += w;
                    for (int k = 0; k < d; ++k) yi[k] += w * (xj[k] + s * (xi[k] - xj[k]));
                }
            }
            mark_row(row_ptr, col_idx, i, flag, 0);
            if (grad)
                for (int k = 0; k < d; ++k) grad[(size_t)r * d + k] = gi[k];
            if (row_loss) row_loss[r] = L;
            if (upper_loss) upper_loss[r] = U;
            if (upper_hits) upper_hits[r] = hits;
            if (zsum) zsum[r] = z;
            if (abs_slope) abs_slope[r] = A;
            if (ysum)
                for (int k = 0; k < d; ++k) ysum[(size_t)r * d + k] = yi[k];
        }
        free(flag);
        free(gi);
        free(yi);
    }
}

/*
 * Whole-graph loss and gradient.
 *   loss      : DL = sum_{i<j} dl(i, j) in bits (summed over rows in index order)
 *   grad      : n x d, may be NULL
 *   edge_hits : number of pairs i<j recognised as edges (must equal m)
 *   row_loss  : n, L_i = sum_{j != i} dl(i, j); may be NULL
 *   abs_slope : n, A_i = sum_{j != i} |d dl(i, j) / d delta|; may be NULL
 */
void oracle_loss_grad(int n, int d, const double *X, const int64_t *row_ptr,
                      const int32_t *col_idx, double mu, double sigma, double *loss, double *grad,
                      int64_t *edge_hits, double *row_loss, double *abs_slope) {
    double *U = (double *)malloc(sizeof(double) * (size_t)n);
    int64_t *H = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    oracle_rows(n, d, X, row_ptr, col_idx, mu, sigma, n, NULL, grad, row_loss, U, H, NULL, NULL,
                abs_slope);
    double total = 0.0;
    int64_t hits = 0;
    for (int i = 0; i < n; ++i) total += U[i], hits += H[i];
    if (loss) *loss = total;
    if (edge_hits) *edge_hits = hits;
    free(U);
    free(H);
}

/*
 * One shard of the all-pairs sum (the split of the pair work over several devices; the paper
 * splits its edge blocks over cores, Sec. III-A).  Pair i < j lies in strip floor(i /
 * strip_rows); with S = ceil(n / strip_rows) strips, strips q and S - 1 - q form strip pair
 * min(q, S - 1 - q), and shard s of G owns the strip pairs p with p mod G == s.
 *   loss      : sum of dl(i, j) over the shard's pairs i < j (rows in index order)
 *   grad      : n x d, row v sums the gradient terms of the shard's pairs that contain v
 *   edge_hits : edges among the shard's pairs
 */
static int shard_owns(int i, int j, int strip_rows, int S, int G, int s) {
    int lo = i < j ? i : j;
    int q = lo / strip_rows;
    int p = q < S - 1 - q ? q : S - 1 - q;
    return p % G == s;
}

/* The same shard for a list of rows only: grad (nrows x d) of rows[r] over the shard's pairs. */
void oracle_rows_shard(int n, int d, const double *X, const int64_t *row_ptr, const int32_t *col_idx,
                       double mu, double sigma, int strip_rows, int nshards, int shard, int nrows,
                       const int64_t *rows, double *grad) {
    const int S = (n + strip_rows - 1) / strip_rows;
#pragma omp parallel
    {
        unsigned char *flag = (unsigned char *)calloc((size_t)n, 1);
#pragma omp for schedule(dynamic, 1)
        for (int r = 0; r < nrows; ++r) {
            const int i = (int)rows[r];
            const double *xi = X + (size_t)i * d;
            mark_row(row_ptr, col_idx, i, flag, 1);
            for (int k = 0; k < d; ++k) grad[(size_t)r * d + k] = 0.0;
            for (int j = 0; j < n; ++j) {
                if (j == i || !shard_owns(i, j, strip_rows, S, nshards, shard)) continue;
                const double *xj = X + (size_t)j * d;
                double r2 = 0.0;
                for (int k = 0; k < d; ++k) r2 += (xi[k] - xj[k]) * (xi[k] - xj[k]);
                double delta = sqrt(r2), dl, d1, d2;
                oracle_pair(delta, flag[j] != 0, mu, sigma, &dl, &d1, &d2);
                double cs = (delta > 0.0) ? d1 / delta : 0.0;
                for (int k = 0; k < d; ++k) grad[(size_t)r * d + k] += cs * (xi[k] - xj[k]);
            }
            mark_row(row_ptr, col_idx, i, flag, 0);
        }
        free(flag);
    }
}

void oracle_loss_grad_shard(int n, int d, const double *X, const int64_t *row_ptr, const int32_t *col_idx,
                            double mu, double sigma, int strip_rows, int nshards, int shard, double *loss,
                            double *grad, int64_t *edge_hits) {
    const int S = (n + strip_rows - 1) / strip_rows;
    double *U = (double *)calloc((size_t)n, sizeof(double));
    int64_t *H = (int64_t *)calloc((size_t)n, sizeof(int64_t));
#pragma omp parallel
    {
        unsigned char *flag = (unsigned char *)calloc((size_t)n, 1);
#pragma omp for schedule(dynamic, 1)
        for (int i = 0; i < n; ++i) {
            const double *xi = X + (size_t)i * d;
            mark_row(row_ptr, col_idx, i, flag, 1);
            for (int j = 0; j < n; ++j) {
                if (j == i || !shard_owns(i, j, strip_rows, S, nshards, shard)) continue;
                const double *xj = X + (size_t)j * d;
                double r2 = 0.0;
                for (int k = 0; k < d; ++k) r2 += (xi[k] - xj[k]) * (xi[k] - xj[k]);
                double delta = sqrt(r2), dl, d1, d2;
                oracle_pair(delta, flag[j] != 0, mu, sigma, &dl, &d1, &d2);
                if (i < j) {
                    U[i] += dl;
                    H[i] += flag[j] != 0;
                }
                double cs = (delta > 0.0) ? d1 / delta : 0.0;
                if (grad)
                    for (int k = 0; k < d; ++k) grad[(size_t)i * d + k] += cs * (xi[k] - xj[k]);
            }
            mark_row(row_ptr, col_idx, i, flag, 0);
        }
        free(flag);
    }
    double total = 0.0;
    int64_t hits = 0;
    for (int i = 0; i < n; ++i) total += U[i], hits += H[i];
    if (loss) *loss = total;
    if (edge_hits) *edge_hits = hits;
    free(U);
    free(H);
}

/* Threads OpenMP will use (for reporting). */
int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/*
 * Slope optimisation (Sec. III-F).  mu stays fixed and sigma is chosen where the derivative
 * of Eq. 2 with respect to sigma vanishes, located by bisection.  With tau = a (delta - mu) /
 * sigma one has d tau / d sigma = -tau / sigma, so
 *   d dl / d sigma = (d dl / d tau)(-tau / sigma) = tau R(tau) / (sigma ln 2),
 * and the condition is F(sigma) = sum_{i<j} tau_ij R(tau_ij) = 0 (F < 0: DL still falls as
 * sigma grows).  The paper evaluates it on histograms of the pair distances, kept separately
 * for edges and non-edges, rather than on the pairs.
 *
 * Histogram layout (the paper gives none; this is the reading): nbins bins uniform in the
 * squared distance on [0, r2_max).  A pair's bin is the integer part of
 * min(r2 * inv_w, nbins - 1), computed in single precision from the single-precision
 * squared distance accumulated coordinate by coordinate with fused multiply-adds, so that a
 * device computing in single precision takes the same decision for every pair.  A bin stands
 * for the distance sqrt((b + 1/2) r2_max / nbins).
 */
void oracle_histogram(int n, int d, const float *X, const int64_t *row_ptr, const int32_t *col_idx,
                      int nbins, float inv_w, uint64_t *hist_all, uint64_t *hist_edge) {
    memset(hist_all, 0, sizeof(uint64_t) * (size_t)nbins);
    memset(hist_edge, 0, sizeof(uint64_t) * (size_t)nbins);
    const float top = (float)(nbins - 1);
#pragma omp parallel
    {
        uint64_t *ha = (uint64_t *)calloc((size_t)nbins, sizeof(uint64_t));
        uint64_t *he = (uint64_t *)calloc((size_t)nbins, sizeof(uint64_t));
        unsigned char *flag = (unsigned char *)calloc((size_t)n, 1);
#pragma omp for schedule(dynamic, 16)
        for (int i = 0; i < n; ++i) {
            mark_row(row_ptr, col_idx, i, flag, 1);
            const float *xi = X + (size_t)i * d;
            for (int j = i + 1; j < n; ++j) {
                const float *xj = X + (size_t)j * d;
                float r2 = 0.0f;
                for (int k = 0; k < d; ++k) {
                    float df = xi[k] - xj[k];
                    r2 = fmaf(df, df, r2);
                }
                int b = (int)fminf(r2 * inv_w, top);
                ha[b] += 1;
                if (flag[j]) he[b] += 1;
            }
            mark_row(row_ptr, col_idx, i, flag, 0);
        }
#pragma omp critical
        for (int b = 0; b < nbins; ++b) {
            hist_all[b] += ha[b];
            hist_edge[b] += he[b];
        }
        free(ha);
        free(he);
        free(flag);
    }
}

/* F(sigma) on the histograms: every bin's edges and non-edges at the bin's distance. */
static double hist_F(double sigma, int nbins, double r2_max, const uint64_t *hist_all,
                     const uint64_t *hist_edge, double mu) {
    double F = 0.0;
    for (int b = 0; b < nbins; ++b) {
        if (!hist_all[b]) continue;
        double delta = sqrt((b + 0.5) * r2_max / nbins);
        double t = (delta - mu) / sigma;          /* tau of a non-edge; an edge has -t */
        double ne = (double)(hist_all[b] - hist_edge[b]);
        double e = (double)hist_edge[b];
        if (ne > 0) F += ne * t * mills_inv(t);
        if (e > 0) F += e * (-t) * mills_inv(-t);
    }
    return F;
}

/* F(sigma) over every pair (exact distances, no histogram). */
static double pairs_F(double sigma, int n, int d, const double *X, const int64_t *row_ptr,
                      const int32_t *col_idx, double mu) {
    double F = 0.0;
#pragma omp parallel reduction(+ : F)
    {
        unsigned char *flag = (unsigned char *)calloc((size_t)n, 1);
#pragma omp for schedule(dynamic, 16)
        for (int i = 0; i < n; ++i) {
            mark_row(row_ptr, col_idx, i, flag, 1);
            for (int j = i + 1; j < n; ++j) {
                double r2 = 0.0;
                for (int k = 0; k < d; ++k) {
                    double df = X[(size_t)i * d + k] - X[(size_t)j * d + k];
                    r2 += df * df;
                }
                double a = flag[j] ? -1.0 : 1.0;
                double t = a * (sqrt(r2) - mu) / sigma;
                F += t * mills_inv(t);
            }
            mark_row(row_ptr, col_idx, i, flag, 0);
        }
        free(flag);
    }
    return F;
}

/* Geometric bisection of F on [lo, hi]; a bracket end is returned when F does not change
 * sign there (the minimum lies on the boundary of the search interval). */
static double bisect_sigma(double (*Fn)(double, const void *), const void *ctx, double lo, double hi,
                           int iters) {
    if (Fn(lo, ctx) >= 0.0) return lo;
    if (Fn(hi, ctx) <= 0.0) return hi;
    for (int it = 0; it < iters; ++it) {
        double s = sqrt(lo * hi);
        if (Fn(s, ctx) < 0.0) lo = s; else hi = s;
    }
    return sqrt(lo * hi);
}

struct hist_ctx { int nbins; double r2_max; const uint64_t *all, *edge; double mu; };
static double hist_fn(double s, const void *c) {
    const struct hist_ctx *h = (const struct hist_ctx *)c;
    return hist_F(s, h->nbins, h->r2_max, h->all, h->edge, h->mu);
}
struct pairs_ctx { int n, d; const double *X; const int64_t *rp; const int32_t *ci; double mu; };
static double pairs_fn(double s, const void *c) {
    const struct pairs_ctx *p = (const struct pairs_ctx *)c;
    return pairs_F(s, p->n, p->d, p->X, p->rp, p->ci, p->mu);
}

double oracle_sigma_hist(int nbins, double r2_max, const uint64_t *hist_all, const uint64_t *hist_edge,
                         double mu, double lo, double hi, int iters) {
    struct hist_ctx c = {nbins, r2_max, hist_all, hist_edge, mu};
    return bisect_sigma(hist_fn, &c, lo, hi, iters);
}

double oracle_sigma_exact(int n, int d, const double *X, const int64_t *row_ptr, const int32_t *col_idx,
                          double mu, double lo, double hi, int iters) {
    struct pairs_ctx c = {n, d, X, row_ptr, col_idx, mu};
    return bisect_sigma(pairs_fn, &c, lo, hi, iters);
}

/*
 * Negative sampling (Sec. III-C, Fig. nonedges, Fig. algo).  Every edge (i, j), i < j, takes
 * part with its own parabola, and with two sampled non-edges: a vertex g with (g, i) not in E
 * for i, and h with (h, j) not in E for j.  One step is Eq. 5 over that multiset of pairs,
 * i.e. x_v <- y_v / z_v with y and z summed over the pairs that contain v; a vertex in no
 * pair keeps its coordinates.
 *
 * Random draws.  The paper's generator is the 32-bit LCG s <- 1103515245 s + 1 (mod 2^32),
 * mapped to a vertex by taking the low 23 bits of s as the mantissa of a float f in [1, 2)
 * and rounding f n - n.  Readings: the float arithmetic is single precision, multiply then
 * subtract; the rounding is floor (round-to-nearest can give n); a draw equal to the vertex
 * itself, outside [0, n), or adjacent to it is rejected and the generator steps again, at
 * most max_tries draws in all (then the sample is dropped: a vertex adjacent to every other
 * has no non-edge).  Each sample owns its generator: the state starts from the upper 32 bits
 * of SplitMix64 (Steele, Lea and Flood 2014) applied to seed + 2 e + side, e the CSR index
 * of the entry (i, j) with i < j, side 0 for i and 1 for j, so the draws do not depend on
 * how the work is divided.
 * samples: int32[2 nnz]; for the entry e with i < j, samples[2e] = g, samples[2e + 1] = h
 * (-1 when dropped); entries with i > j hold -1.
 */
static uint64_t splitmix64(uint64_t x) {
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

/* Is (a, b) an edge: binary search in a's sorted CSR row. */
static int is_edge(const int64_t *row_ptr, const int32_t *col_idx, int a, int b) {
    int64_t lo = row_ptr[a], hi = row_ptr[a + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (col_idx[mid] < b) lo = mid + 1; else hi = mid;
    }
    return lo < row_ptr[a + 1] && col_idx[lo] == b;
}

static int draw_non_neighbour(int v, int n, uint32_t state, int max_tries, const int64_t *row_ptr,
                              const int32_t *col_idx) {
    const float nf = (float)n;
    for (int t = 0; t < max_tries; ++t) {
        state = 1103515245u * state + 1u;
        uint32_t bits = 0x3f800000u | (state & 0x7fffffu);
        float f;
        memcpy(&f, &bits, sizeof(f));
        volatile float prod = f * nf;  /* separate rounding of the product and the difference */
        float u = prod - nf;
        int c = (int)floorf(u);
        if (c < 0 || c >= n || c == v) continue;
        if (is_edge(row_ptr, col_idx, v, c)) continue;
        return c;
    }
    return -1;
}

void oracle_sample_pairs(int n, const int64_t *row_ptr, const int32_t *col_idx, uint64_t seed, int max_tries,
                         int32_t *samples) {
    int64_t nnz = row_ptr[n];
    for (int i = 0; i < n; ++i) {
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            int j = col_idx[e];
            samples[2 * e] = samples[2 * e + 1] = -1;
            if (i >= j) continue;
            uint32_t s0 = (uint32_t)(splitmix64(seed + 2 * (uint64_t)e) >> 32);
            uint32_t s1 = (uint32_t)(splitmix64(seed + 2 * (uint64_t)e + 1) >> 32);
            samples[2 * e] = draw_non_neighbour(i, n, s0, max_tries, row_ptr, col_idx);
            samples[2 * e + 1] = draw_non_neighbour(j, n, s1, max_tries, row_ptr, col_idx);
        }
    }
    (void)nnz;
}

/* Adds one pair's parabola (Eq. 3-4) to y and z of both ends, and its dl to *loss. */
static void add_pair(int d, const double *X, int a, int b, int edge, double mu, double sigma, double *Y,
                     double *Z, double *loss) {
    double r2 = 0.0;
    for (int k = 0; k < d; ++k) {
        double diff = X[(size_t)a * d + k] - X[(size_t)b * d + k];
        r2 += diff * diff;
    }
    double delta = sqrt(r2), dl, d1, d2;
    oracle_pair(delta, edge, mu, sigma, &dl, &d1, &d2);
    double w = 0.5 * d2;
    double dij = delta - d1 / (2.0 * w);
    double s = (delta > 0.0) ? dij / delta : 0.0;
    for (int k = 0; k < d; ++k) {
        double xa = X[(size_t)a * d + k], xb = X[(size_t)b * d + k];
        Y[(size_t)a * d + k] += w * (xb + s * (xa - xb));
        Y[(size_t)b * d + k] += w * (xa + s * (xb - xa));
    }
    Z[a] += w;
    Z[b] += w;
    *loss += dl;
}

/* One negative-sampled weighted-majorization step from X (FP64): X_new, the dl summed over
 * the pairs used (edges and samples), and the samples drawn. */
void oracle_sampled_step(int n, int d, const double *X, const int64_t *row_ptr, const int32_t *col_idx,
                         double mu, double sigma, uint64_t seed, int max_tries, double *X_new,
                         double *loss_sampled, int32_t *samples) {
    oracle_sample_pairs(n, row_ptr, col_idx, seed, max_tries, samples);
    double *Y = (double *)calloc((size_t)n * d, sizeof(double));
    double *Z = (double *)calloc((size_t)n, sizeof(double));
    double loss = 0.0;
    for (int i = 0; i < n; ++i) {
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            int j = col_idx[e];
            if (i >= j) continue;
            add_pair(d, X, i, j, 1, mu, sigma, Y, Z, &loss);
            if (samples[2 * e] >= 0) add_pair(d, X, i, samples[2 * e], 0, mu, sigma, Y, Z, &loss);
            if (samples[2 * e + 1] >= 0) add_pair(d, X, j, samples[2 * e + 1], 0, mu, sigma, Y, Z, &loss);
        }
    }
    for (int v = 0; v < n; ++v)
        for (int k = 0; k < d; ++k)
            X_new[(size_t)v * d + k] = (Z[v] > 0.0) ? Y[(size_t)v * d + k] / Z[v] : X[(size_t)v * d + k];
    if (loss_sampled) *loss_sampled = loss;
    free(Y);
    free(Z);
}
