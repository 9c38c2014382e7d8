/*
 * CPU FP64 reference ("oracle") for exact Reverse k-Maximum Inner Product Search.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link, load or
 * call this file: only the test suite, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code, header, table or constant with the GPU
 * library; both sides receive the same seeded inputs and nothing else.
 *
 * It is deliberately plain and slow: every result is computed straight from its
 * definition, one pair at a time, in IEEE double precision.
 *
 *  - Definition 1 (RkMIPS): user u is in the answer for query q and k iff q is
 *    among the k largest inner products of u over P united with {q}.  With the
 *    tie reading "q wins ties" (the query algorithms prune only on a strict "<",
 *    Alg. 5 and Alg. 2) this is:  #{p in P : s(u,p) > s(u,q)} < k, equivalently
 *    s(u,q) >= lambda_u^(k), the k-th largest s(u,p) over P (-inf when k > n).
 *  - s(u,x) is the canonical FP64 inner product (the paper fixes no precision):
 *      FP32 / BF16 storage: acc = +0; for i = 0..d-1: acc = acc + u_i * x_i
 *        (every product of two FP32 values is exact in FP64, so only the sums
 *        round, in index order);
 *      FP8 e4m3 storage with per-vector scales:  S = sum_i c_ui * c_xi over the
 *        decoded codes (exact in FP64 in any order: multiples of 2^-18 below 2^26),
 *        then s = (scale_u * scale_x) * S  (the scale product is exact; one rounding).
 *  - Item norms and order (Alg. 4, norms and sort; Alg. 1, first step):
 *        n2(p) = sum_i p_i^2 in the same canonical way; items sorted by n2
 *        descending, equal keys by ascending index.
 *  - SA-ALSH indexing (Alg. 1): norm partitions, centroids, radii, the
 *    shifting-invariant item transform (Eqn. 6) and sign-random-projection codes
 *    (Eqn. 1) for a given projection matrix; user codes from Eqn. 7.
 *  - SA-ALSH query (Alg. 2) for one (user, query, k), with the collision-count
 *    candidate reading stated at saalsh_decide.
 *
 * Build: gcc -O2 -fopenmp -fno-fast-math -ffp-contract=off -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_F32 = 0, ORC_BF16 = 1, ORC_FP8 = 2 };

/* ---------------------------------------------------------------- storage decoding */

/* BF16: the 16 stored bits are the upper half of an FP32 pattern. */
static double bf16_value(uint16_t bits)
{
    uint32_t w = (uint32_t)bits << 16;
    float f;
    memcpy(&f, &w, sizeof f);
    return (double)f;
}

/* FP8 e4m3 (OCP e4m3fn): sign | 4 exponent bits (bias 7) | 3 mantissa bits;
 * exponent 0 is subnormal (m * 2^-9); 0x7F/0xFF are NaN; no infinities. */
double orc_e4m3_value(uint8_t code)
{
    int sign = code >> 7, e = (code >> 3) & 15, mnt = code & 7;
    double v;
    if (e == 15 && mnt == 7) return NAN;
    if (e == 0) v = ldexp((double)mnt, -9);
    else        v = ldexp((double)(8 + mnt), e - 10);
    return sign ? -v : v;
}

/* Element i of row r of a stored matrix, as the exact double it denotes
 * (for FP8 this is the unscaled code value). */
static double elem(const void *base, int dtype, int64_t r, int d, int i)
{
    switch (dtype) {
    case ORC_F32:  return (double)((const float *)base)[r * d + i];
    case ORC_BF16: return bf16_value(((const uint16_t *)base)[r * d + i]);
    default:       return orc_e4m3_value(((const uint8_t *)base)[r * d + i]);
    }
}

static double row_scale(const float *scales, int dtype, int64_t r)
{
    return dtype == ORC_FP8 ? (double)scales[r] : 1.0;
}

/* ------------------------------------------------------------------ canonical score */

/* s(a_row, b_row): the canonical FP64 inner product defined in the header. */
double orc_score(int dtype, int d,
                 const void *A, const float *a_scales, int64_t ra,
                 const void *B, const float *b_scales, int64_t rb)
{
    double acc = 0.0;
    for (int i = 0; i < d; i++)
        acc = acc + elem(A, dtype, ra, d, i) * elem(B, dtype, rb, d, i);
    if (dtype == ORC_FP8)
        acc = (row_scale(a_scales, dtype, ra) * row_scale(b_scales, dtype, rb)) * acc;
    return acc;
}

/* n2(x) = <x,x> in the canonical way. */
double orc_norm2(int dtype, int d, const void *X, const float *scales, int64_t r)
{
    return orc_score(dtype, d, X, scales, r, X, scales, r);
}

/* ------------------------------------------------------- lambda table (Def. 1, Alg. 4) */

static int cmp_desc(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x < y) - (x > y);
}

/* The rows of a stored matrix as the exact doubles they denote (FP8: unscaled code
 * values), decoded once: rows[r*d + i] = elem(X, r, i).  NULL on allocation failure. */
static double *decode_rows(const void *X, int dtype, const int64_t *row_idx, int64_t nrows, int d)
{
    double *out = (double *)malloc(sizeof(double) * (size_t)(nrows > 0 ? nrows : 1) * (size_t)d);
    if (!out) return NULL;
    for (int64_t t = 0; t < nrows; t++) {
        int64_t r = row_idx ? row_idx[t] : t;
        for (int i = 0; i < d; i++) out[t * d + i] = elem(X, dtype, r, d, i);
    }
    return out;
}

/* The canonical score of two decoded rows: index-order sum, then the scale product for
 * FP8 (the same arithmetic as orc_score). */
static double dot_decoded(int dtype, int d, const double *a, double sa, const double *b, double sb)
{
    double acc = 0.0;
    for (int i = 0; i < d; i++)
        acc = acc + a[i] * b[i];
    if (dtype == ORC_FP8)
        acc = (sa * sb) * acc;
    return acc;
}

/* lambda[j*m_sel + t] = (j+1)-th largest s(u,p) over all p in P, for the user
 * u = user_idx[t] (or t when user_idx is NULL), j < k_max; -inf for j >= n. */
int orc_lambda(int dtype, int d,
               const void *P, const float *p_scales, int64_t n,
               const void *U, const float *u_scales,
               const int64_t *user_idx, int64_t m_sel,
               int k_max, double *lambda, int nthreads)
{
    int bad = 0;
    double *Pd = decode_rows(P, dtype, NULL, n, d);
    if (!Pd) return -1;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1) reduction(| : bad)
    {
        double *buf = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        double *ur = (double *)malloc(sizeof(double) * (size_t)d);
        if (!buf || !ur) bad = 1;
#pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < m_sel; t++) {
            if (!buf || !ur) continue;
            int64_t u = user_idx ? user_idx[t] : t;
            for (int i = 0; i < d; i++) ur[i] = elem(U, dtype, u, d, i);
            double su = row_scale(u_scales, dtype, u);
            for (int64_t p = 0; p < n; p++)
                buf[p] = dot_decoded(dtype, d, ur, su, Pd + p * d, row_scale(p_scales, dtype, p));
            qsort(buf, (size_t)n, sizeof(double), cmp_desc);
            for (int j = 0; j < k_max; j++)
                lambda[(int64_t)j * m_sel + t] = j < n ? buf[j] : -INFINITY;
        }
        free(buf);
        free(ur);
    }
    free(Pd);
    return bad ? -1 : 0;
}

/* member[qi*m_sel + t] = 1 iff s(u,q) >= lambda_u^(k_q)  (u = user_idx[t]). */
int orc_member(int dtype, int d,
               const void *U, const float *u_scales,
               const int64_t *user_idx, int64_t m_sel,
               const void *Q, const float *q_scales, int64_t nq, const int32_t *ks,
               const double *lambda, int k_max, uint8_t *member, int nthreads)
{
    for (int64_t qi = 0; qi < nq; qi++)
        if (ks[qi] < 1 || ks[qi] > k_max) return -1;
    double *Ud = decode_rows(U, dtype, user_idx, m_sel, d);
    double *Qd = decode_rows(Q, dtype, NULL, nq, d);
    if (!Ud || !Qd) { free(Ud); free(Qd); return -2; }
#pragma omp parallel for num_threads(nthreads > 0 ? nthreads : 1) schedule(dynamic, 4)
    for (int64_t qi = 0; qi < nq; qi++) {
        int k = ks[qi];
        double sq = row_scale(q_scales, dtype, qi);
        for (int64_t t = 0; t < m_sel; t++) {
            int64_t u = user_idx ? user_idx[t] : t;
            double s = dot_decoded(dtype, d, Ud + t * d, row_scale(u_scales, dtype, u), Qd + qi * d, sq);
            member[qi * m_sel + t] = s >= lambda[(int64_t)(k - 1) * m_sel + t];
        }
    }
    free(Ud);
    free(Qd);
    return 0;
}

/* beats[qi*m_sel + t] = #{p in P : s(u,p) > s(u,q)}: the direct count form of
 * Definition 1 (q is in u's top-k over P with q iff this count is < k). */
int orc_count_beating(int dtype, int d,
                      const void *P, const float *p_scales, int64_t n,
                      const void *U, const float *u_scales,
                      const int64_t *user_idx, int64_t m_sel,
                      const void *Q, const float *q_scales, int64_t nq,
                      int64_t *beats, int nthreads)
{
#pragma omp parallel for num_threads(nthreads > 0 ? nthreads : 1) schedule(dynamic, 4)
    for (int64_t t = 0; t < m_sel; t++) {
        int64_t u = user_idx ? user_idx[t] : t;
        for (int64_t qi = 0; qi < nq; qi++) {
            double sq = orc_score(dtype, d, U, u_scales, u, Q, q_scales, qi);
            int64_t c = 0;
            for (int64_t p = 0; p < n; p++)
                c += orc_score(dtype, d, U, u_scales, u, P, p_scales, p) > sq;
            beats[qi * m_sel + t] = c;
        }
    }
    return 0;
}

/* ------------------------------------------------------------ item order (Alg. 4 / 1) */

static const double *g_sort_keys;
static int cmp_order(const void *a, const void *b)
{
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    double x = g_sort_keys[i], y = g_sort_keys[j];
    if (x > y) return -1;
    if (x < y) return 1;
    return (i > j) - (i < j);
}

/* norm2[p] = n2(p); order = item indices by n2 descending, ties by index. */
int orc_item_order(int dtype, int d, const void *P, const float *p_scales, int64_t n,
                   double *norm2, int64_t *order)
{
    for (int64_t p = 0; p < n; p++) {
        norm2[p] = orc_norm2(dtype, d, P, p_scales, p);
        order[p] = p;
    }
    g_sort_keys = norm2;
    qsort(order, (size_t)n, sizeof(int64_t), cmp_order);
    return 0;
}

/* ------------------------------------------------------------ SA-ALSH indexing (Alg. 1) */

/* Norm partitions over the items taken in `order` (descending n2).  Partition j
 * starts at the first unassigned item, with M_j^2 = its n2, and takes items while
 * n2(p) > (b*b) * M_j^2 (the squared form of ||p|| > b*M_j, evaluated in FP64 with
 * b*b exact).  When M_j = 0 the loop of Alg. 1 would not advance; the remaining
 * (zero-norm) items then form one last partition.
 * part_start[j] .. part_start[j+1] index into `order`; returns t. */
int orc_partitions(const double *norm2, const int64_t *order, int64_t n, float b,
                   int64_t *part_start, int max_parts)
{
    double bb = (double)b * (double)b;
    int64_t i = 0;
    int t = 0;
    while (i < n) {
        if (t >= max_parts) return -1;
        part_start[t++] = i;
        double M2 = norm2[order[i]];
        if (M2 == 0.0) { i = n; break; }
        double thr = bb * M2;
        while (i < n && norm2[order[i]] > thr) i++;
    }
    part_start[t] = n;
    return t;
}

/* For each partition j: centroid c_j (mean, FP64 sum in `order` sequence divided by
 * |S_j|), radius R_j = max ||p - c_j||, transformed item
 * I(p, c_j) = [p - c_j ; sqrt(max(0, R_j^2 - ||p - c_j||^2))] (Eqn. 6) and its K-bit
 * code: bit h = (<I(p,c_j), a_h> >= 0) with a_h column h of the (d+1) x K matrix A
 * (sgn(0) taken as +1).  Codes are stored per ORIGINAL item index, K/32 words per
 * item, bit h in word h/32 at position h%32.  centroid is [t x d], radius [t]. */
int orc_saalsh_index(int dtype, int d, const void *P, const float *p_scales, int64_t n,
                     const int64_t *order, const int64_t *part_start, int t,
                     const float *A, int K, double *centroid, double *radius,
                     uint32_t *codes)
{
    int W = K / 32;
    double *x = (double *)malloc(sizeof(double) * (size_t)(d + 1));
    if (!x) return -1;
    for (int j = 0; j < t; j++) {
        int64_t s0 = part_start[j], s1 = part_start[j + 1];
        double *c = centroid + (int64_t)j * d;
        for (int i = 0; i < d; i++) {
            double acc = 0.0;
            for (int64_t s = s0; s < s1; s++)
                acc = acc + row_scale(p_scales, dtype, order[s]) * elem(P, dtype, order[s], d, i);
            c[i] = acc / (double)(s1 - s0);
        }
        double R2 = 0.0;
        for (int64_t s = s0; s < s1; s++) {
            double r2 = 0.0;
            for (int i = 0; i < d; i++) {
                double v = row_scale(p_scales, dtype, order[s]) * elem(P, dtype, order[s], d, i) - c[i];
                r2 = r2 + v * v;
            }
            if (r2 > R2) R2 = r2;
        }
        radius[j] = sqrt(R2);
        for (int64_t s = s0; s < s1; s++) {
            int64_t p = order[s];
            double r2 = 0.0;
            for (int i = 0; i < d; i++) {
                x[i] = row_scale(p_scales, dtype, p) * elem(P, dtype, p, d, i) - c[i];
                r2 = r2 + x[i] * x[i];
            }
            double rest = R2 - r2;
            x[d] = rest > 0.0 ? sqrt(rest) : 0.0;
            for (int w = 0; w < W; w++) codes[p * W + w] = 0u;
            for (int h = 0; h < K; h++) {
                double pr = 0.0;
                for (int i = 0; i <= d; i++) pr = pr + x[i] * (double)A[(int64_t)i * K + h];
                if (pr >= 0.0) codes[p * W + h / 32] |= 1u << (h % 32);
            }
        }
    }
    free(x);
    return 0;
}

/* User codes (Eqn. 7): U(u) = [R_j/||u|| * u ; 0]; the positive factor does not
 * change signs, so bit h = (<u, a_h[0..d-1]> >= 0) for every partition. */
int orc_user_codes(int dtype, int d, const void *U, const float *u_scales, int64_t m,
                   const float *A, int K, uint32_t *codes)
{
    int W = K / 32;
    for (int64_t u = 0; u < m; u++) {
        for (int w = 0; w < W; w++) codes[u * W + w] = 0u;
        for (int h = 0; h < K; h++) {
            double pr = 0.0;
            for (int i = 0; i < d; i++)
                pr = pr + row_scale(u_scales, dtype, u) * elem(U, dtype, u, d, i) * (double)A[(int64_t)i * K + h];
            if (pr >= 0.0) codes[u * W + h / 32] |= 1u << (h % 32);
        }
    }
    return 0;
}

/* ---------------------------------------------------------------- SA-ALSH query (Alg. 2) */

static int popcount32(uint32_t v)
{
    int c = 0;
    while (v) { c += (int)(v & 1u); v >>= 1; }
    return c;
}

/* Alg. 2 for one user u, query q and k.  Partitions are visited in order (M_j
 * descending).  mu_j = M_j * ||u|| (M_j = sqrt of the partition's first n2,
 * ||u|| = sqrt(n2(u))).  If phi > mu_j the answer is yes.  Otherwise the
 * SimHash probe of S_j returns the ceil(beta * |S_j|) items with the largest
 * collision count K - popcount(code_u XOR code_p) (equal counts: earlier in
 * `order` first) -- the reading of "K hash tables" as one K-bit code per item and
 * of probed buckets as a fraction beta of the partition.  phi is then the k-th
 * largest s(u,p) over all candidates so far (-inf while fewer than k), and the
 * answer is no when s(u,q) < phi.  After the last partition the answer is yes.
 * init[0 .. n_init) (may be empty): scores that are candidates before the first
 * partition -- in SAH (Alg. 5) the scores of u on the items of P' that Alg. 4 set
 * aside, whose index covers P \ P' only; phi starts as their k-th largest.
 * Returns 1 (yes) or 0 (no); *phi_out receives the final phi. */
int orc_saalsh_decide(int dtype, int d,
                      const void *P, const float *p_scales, const double *norm2,
                      const int64_t *order, const int64_t *part_start, int t,
                      const uint32_t *item_codes, const uint32_t *user_code, int K,
                      float beta, const void *U, const float *u_scales, int64_t u,
                      const void *Q, const float *q_scales, int64_t qi, int k,
                      const double *init, int64_t n_init, double *phi_out)
{
    int W = K / 32;
    int64_t n = part_start[t];
    double *cand = (double *)malloc(sizeof(double) * (size_t)(n + n_init > 0 ? n + n_init : 1));
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int *col = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    if (!cand || !idx || !col) { free(cand); free(idx); free(col); return -1; }
    int64_t nc = 0;
    double phi = -INFINITY;
    for (int64_t i = 0; i < n_init; i++) cand[nc++] = init[i];
    if (nc >= k) {
        double *tmp = (double *)malloc(sizeof(double) * (size_t)nc);
        if (!tmp) { free(cand); free(idx); free(col); return -1; }
        memcpy(tmp, cand, sizeof(double) * (size_t)nc);
        qsort(tmp, (size_t)nc, sizeof(double), cmp_desc);
        phi = tmp[k - 1];
        free(tmp);
    }
    double unorm = sqrt(orc_norm2(dtype, d, U, u_scales, u));
    double suq = orc_score(dtype, d, U, u_scales, u, Q, q_scales, qi);
    int ans = 1;
    for (int j = 0; j < t; j++) {
        int64_t s0 = part_start[j], s1 = part_start[j + 1], sz = s1 - s0;
        double mu = sqrt(norm2[order[s0]]) * unorm;
        if (phi > mu) { ans = 1; break; }
        /* collision counts, then a stable selection of the ceil(beta*sz) largest */
        for (int64_t s = 0; s < sz; s++) {
            int64_t p = order[s0 + s];
            int diff = 0;
            for (int w = 0; w < W; w++) diff += popcount32(item_codes[p * W + w] ^ user_code[w]);
            col[s] = K - diff;
            idx[s] = s;
        }
        int64_t take = (int64_t)ceil((double)beta * (double)sz);
        if (take > sz) take = sz;
        for (int64_t a = 0; a < take; a++) {          /* selection sort prefix */
            int64_t best = a;
            for (int64_t b2 = a + 1; b2 < sz; b2++)
                if (col[idx[b2]] > col[idx[best]] ||
                    (col[idx[b2]] == col[idx[best]] && idx[b2] < idx[best])) best = b2;
            int64_t tmp = idx[a]; idx[a] = idx[best]; idx[best] = tmp;
            cand[nc++] = orc_score(dtype, d, U, u_scales, u, P, p_scales, order[s0 + idx[a]]);
        }
        if (nc >= k) {
            double *tmp = (double *)malloc(sizeof(double) * (size_t)nc);
            if (!tmp) { ans = -1; break; }
            memcpy(tmp, cand, sizeof(double) * (size_t)nc);
            qsort(tmp, (size_t)nc, sizeof(double), cmp_desc);
            phi = tmp[k - 1];
            free(tmp);
        }
        if (suq < phi) { ans = 0; break; }
    }
    if (phi_out) *phi_out = phi;
    free(cand); free(idx); free(col);
    return ans;
}
