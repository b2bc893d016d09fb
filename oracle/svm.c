/*
 * Order categories by linear support vector machines -- TEST INFRASTRUCTURE
 * ONLY (the CPU oracle of the GPU path; never linked into the product).
 *
 * Section 5, subroutine 5: each order belongs to a category of orders, and an
 * SVM (Cortes and Vapnik 1995) configures the categories from the outputs of
 * the subroutines before it; since the composition of orders changes over
 * time, the SVM is updated continuously from a collection of the most recent
 * orders, newer data replacing older.
 *
 * Readings (the paper gives no features, model or training rule):
 *   - the features of an order are the shares of its lines in each product
 *     category (the categories of Subproblem 3, e.g. K-means classes):
 *     x[c] = (lines in category c) / (lines of the order);
 *   - one linear SVM per category of orders against the rest: hinge loss
 *     plus lambda / 2 times the squared norm of the weights, the bias taken
 *     as the weight of a constant feature 1; trained on the window by
 *     full-batch subgradient steps with the step sizes of Pegasos
 *     (Shalev-Shwartz et al. 2007), eta_t = 1 / (lambda t), t counting every
 *     step since creation;
 *   - an order is assigned the category of the largest score (ties: the
 *     lower category).
 * Every sum runs in a fixed order (features in index order, samples from
 * the oldest), in IEEE double, one operation at a time (built with
 * -ffp-contract=off).
 */
#include <stdint.h>
#include <stdlib.h>

/* x[o * F + c]: the share of order o's lines whose SKU is in category c;
 * lines naming a SKU outside [0, n_skus) or a category outside [0, F) are
 * counted in the order's length only. */
void orc_order_features(int32_t n_orders, const int32_t *off, const int32_t *skus, const int32_t *sku_cat,
                        int32_t n_skus, int32_t F, double *x)
{
    for (int32_t o = 0; o < n_orders; o++) {
        double *row = x + (int64_t)o * F;
        for (int32_t c = 0; c < F; c++) row[c] = 0.0;
        const int32_t len = off[o + 1] - off[o];
        for (int32_t l = off[o]; l < off[o + 1]; l++) {
            const int32_t s = skus[l];
            if (s < 0 || s >= n_skus) continue;
            const int32_t c = sku_cat[s];
            if (c < 0 || c >= F) continue;
            row[c] = row[c] + 1.0;
        }
        for (int32_t c = 0; c < F; c++) row[c] = row[c] / (double)len;
    }
}

/* Score of sample x under class k's weights w[k * (F + 1) ..] (bias last). */
static double orc_svm_score(const double *w, const double *x, int32_t F)
{
    double s = 0.0;
    for (int32_t f = 0; f < F; f++) s = s + w[f] * x[f];
    return s + w[F];
}

/* `iters` full-batch subgradient steps on the n samples x[n][F] with labels
 * in [0, K) (other labels count as negatives for every class), from the
 * weights w[K][F + 1] (in and out), steps numbered t0 + 1, t0 + 2, ...
 * Returns 0, or 3 when memory runs out. */
int orc_svm_train(int32_t n, int32_t F, int32_t K, const double *x, const int32_t *label, double lambda, int64_t t0,
                  int32_t iters, double *w)
{
    int8_t *coef = (int8_t *)malloc((size_t)(n > 0 ? n : 1) * (size_t)K);
    if (!coef) return 3;
    for (int32_t it = 0; it < iters; it++) {
        const double t = (double)(t0 + it + 1);
        const double eta = 1.0 / (lambda * t);
        /* the samples inside the margin at the current weights */
        for (int32_t i = 0; i < n; i++)
            for (int32_t k = 0; k < K; k++) {
                const double y = label[i] == k ? 1.0 : -1.0;
                const double s = orc_svm_score(w + (int64_t)k * (F + 1), x + (int64_t)i * F, F);
                coef[(int64_t)i * K + k] = (int8_t)(y * s < 1.0 ? (label[i] == k ? 1 : -1) : 0);
            }
        /* w_k <- w_k - eta (lambda w_k - (1/n) sum y_i x_i), the bias with the
         * constant feature 1 */
        for (int32_t k = 0; k < K; k++) {
            double *wk = w + (int64_t)k * (F + 1);
            for (int32_t f = 0; f < F; f++) {
                double g = 0.0;
                for (int32_t i = 0; i < n; i++) g = g + (double)coef[(int64_t)i * K + k] * x[(int64_t)i * F + f];
                wk[f] = wk[f] - eta * (lambda * wk[f] - g / (double)n);
            }
            double gb = 0.0;
            for (int32_t i = 0; i < n; i++) gb = gb + (double)coef[(int64_t)i * K + k];
            wk[F] = wk[F] - eta * (lambda * wk[F] - gb / (double)n);
        }
    }
    free(coef);
    return 0;
}

/* Class of each of n samples: the largest score, ties to the lower class. */
void orc_svm_predict(int64_t n, int32_t F, int32_t K, const double *x, const double *w, int32_t *cls)
{
    for (int64_t i = 0; i < n; i++) {
        int32_t best = 0;
        double bs = orc_svm_score(w, x + i * F, F);
        for (int32_t k = 1; k < K; k++) {
            const double s = orc_svm_score(w + (int64_t)k * (F + 1), x + i * F, F);
            if (s > bs) {
                bs = s;
                best = k;
            }
        }
        cls[i] = best;
    }
}
