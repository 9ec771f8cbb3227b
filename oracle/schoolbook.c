/*
 * ORACLE -- test infrastructure only.  Not part of the product path.
 *
 * Plain schoolbook product of two dense polynomials of Z[y].
 *
 * Definition followed: the problem statement of Section 1 (product c = a*b of
 * a(y), b(y) in Z[y]) and the coefficient form given at the start of Section 2,
 * c_i = sum over l + m = i of a_l * b_m.  Coefficients are stored as in
 * Section 2.3 (one fixed-width two's complement block of ceil(N/64) 64-bit
 * words per coefficient, coefficient i at words [i*w, (i+1)*w)), with N the
 * two's complement bound of Relation (definingN).
 *
 * This file shares no code with the GPU library: it has its own decoder, its
 * own multi-word multiply and its own encoder.  Nothing here knows about limbs,
 * primes or transforms.
 *
 * Encoding: word 0 is least significant.  Only bits [0, N) are read; the value
 * is sign-extended from bit N-1.  The output coefficient is written as wc words
 * of two's complement (the exact value reduced mod 2^(64*wc); callers size wc
 * so that nothing is lost).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

/* Decode one coefficient: magnitude into mag[0..w) and return 1 if negative. */
static int decode_coeff(const uint64_t *src, int32_t N, uint64_t *mag, int32_t w)
{
    /* sign-extend from bit N-1 into a private copy */
    int32_t top = (N - 1) / 64;           /* word that holds bit N-1 */
    int32_t bit = (N - 1) % 64;
    uint64_t tmp[w];
    for (int32_t k = 0; k < w; ++k) tmp[k] = src[k];
    int neg = (int)((tmp[top] >> bit) & 1u);
    if (bit < 63) {
        uint64_t keep = (((uint64_t)1) << (bit + 1)) - 1;
        tmp[top] = neg ? (tmp[top] | ~keep) : (tmp[top] & keep);
    }
    for (int32_t k = top + 1; k < w; ++k) tmp[k] = neg ? ~(uint64_t)0 : 0;
    if (!neg) {
        for (int32_t k = 0; k < w; ++k) mag[k] = tmp[k];
    } else {
        /* magnitude = (~tmp) + 1 */
        uint64_t carry = 1;
        for (int32_t k = 0; k < w; ++k) {
            uint64_t v = ~tmp[k];
            uint64_t s = v + carry;
            carry = (carry && s == 0) ? 1 : 0;
            mag[k] = s;
        }
    }
    return neg;
}

/* acc[0..wacc) += x[0..wx) * y[0..wy), all unsigned. */
static void mac(uint64_t *acc, int32_t wacc, const uint64_t *x, int32_t wx,
                const uint64_t *y, int32_t wy)
{
    for (int32_t u = 0; u < wx; ++u) {
        if (x[u] == 0) continue;
        uint64_t carry = 0;
        int32_t v;
        for (v = 0; v < wy; ++v) {
            u128 t = (u128)x[u] * y[v] + acc[u + v] + carry;
            acc[u + v] = (uint64_t)t;
            carry = (uint64_t)(t >> 64);
        }
        for (int32_t k = u + v; carry && k < wacc; ++k) {
            u128 t = (u128)acc[k] + carry;
            acc[k] = (uint64_t)t;
            carry = (uint64_t)(t >> 64);
        }
    }
}

/* One output coefficient c_i = sum_{l+m=i} a_l b_m, written as wc words. */
static void one_coeff(int64_t i,
                      const uint64_t *amag, const unsigned char *aneg, int64_t da, int32_t wa,
                      const uint64_t *bmag, const unsigned char *bneg, int64_t db, int32_t wb,
                      uint64_t *out, int32_t wc, uint64_t *pos, uint64_t *neg, int32_t wacc)
{
    memset(pos, 0, sizeof(uint64_t) * (size_t)wacc);
    memset(neg, 0, sizeof(uint64_t) * (size_t)wacc);
    int64_t lo = i - (db - 1) > 0 ? i - (db - 1) : 0;
    int64_t hi = i < da - 1 ? i : da - 1;
    for (int64_t l = lo; l <= hi; ++l) {
        int64_t m = i - l;
        uint64_t *dst = (aneg[l] ^ bneg[m]) ? neg : pos;
        mac(dst, wacc, amag + (size_t)l * wa, wa, bmag + (size_t)m * wb, wb);
    }
    /* c = pos - neg in two's complement of wacc words, then resize to wc words */
    uint64_t borrow = 0;
    for (int32_t k = 0; k < wacc; ++k) {
        uint64_t x = pos[k], y = neg[k];
        uint64_t d = x - y - borrow;
        borrow = (x < y) || (x == y && borrow) ? 1 : 0;
        pos[k] = d;
    }
    uint64_t fill = (pos[wacc - 1] >> 63) ? ~(uint64_t)0 : 0;
    for (int32_t k = 0; k < wc; ++k) out[k] = k < wacc ? pos[k] : fill;
}

static int prepare(const uint64_t *src, int64_t d, int32_t N, int32_t w,
                   uint64_t **mag, unsigned char **neg)
{
    *mag = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(d > 0 ? d : 1) * (size_t)w);
    *neg = (unsigned char *)malloc((size_t)(d > 0 ? d : 1));
    if (!*mag || !*neg) return -1;
    for (int64_t l = 0; l < d; ++l)
        (*neg)[l] = (unsigned char)decode_coeff(src + (size_t)l * w, N, *mag + (size_t)l * w, w);
    return 0;
}

/*
 * Compute the output coefficients listed in rows[0..nrows) (or all da+db-1 of
 * them when rows == NULL) into c: output row r (the r-th listed index) is at
 * c + r*wc.  Returns 0, or -1 on bad arguments / allocation failure.
 */
int oracle_polymul_rows(const uint64_t *a, int64_t da, int32_t Na,
                        const uint64_t *b, int64_t db, int32_t Nb,
                        uint64_t *c, int32_t wc,
                        const int64_t *rows, int64_t nrows, int nthreads)
{
    if (da < 0 || db < 0 || Na < 1 || Nb < 1 || wc < 1) return -1;
    if (da == 0 || db == 0) return 0;
    int32_t wa = (Na + 63) / 64, wb = (Nb + 63) / 64;
    int64_t nout = da + db - 1;
    if (!rows) nrows = nout;
    uint64_t *amag, *bmag;
    unsigned char *aneg, *bneg;
    if (prepare(a, da, Na, wa, &amag, &aneg) || prepare(b, db, Nb, wb, &bmag, &bneg)) return -1;
    /* |c_i| < min(da,db) * 2^(Na+Nb-2); one spare word for the count and one for the sign */
    int32_t wacc = wa + wb + 2;
    int bad = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
    {
        uint64_t *pos = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)wacc);
        uint64_t *ngv = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)wacc);
        if (!pos || !ngv) {
            bad = 1;
        } else {
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
            for (int64_t r = 0; r < nrows; ++r) {
                int64_t i = rows ? rows[r] : r;
                if (i < 0 || i >= nout) { bad = 1; continue; }
                one_coeff(i, amag, aneg, da, wa, bmag, bneg, db, wb,
                          c + (size_t)r * wc, wc, pos, ngv, wacc);
            }
        }
        free(pos);
        free(ngv);
    }
    free(amag); free(aneg); free(bmag); free(bneg);
    return bad ? -1 : 0;
}

int oracle_polymul(const uint64_t *a, int64_t da, int32_t Na,
                   const uint64_t *b, int64_t db, int32_t Nb,
                   uint64_t *c, int32_t wc, int nthreads)
{
    return oracle_polymul_rows(a, da, Na, b, db, Nb, c, wc, NULL, 0, nthreads);
}

/*
 * The same product reduced modulo q: c_i mod q = sum_{l+m=i} (a_l mod q)(b_m mod q)
 * mod q, for every i in [0, da+db-1), written as residues in [0, q) to c[i].
 * This is the definition of the product (Section 1, Section 2's c_i) taken in
 * Z/qZ; it serves to check every coefficient of a product far too large for the
 * exact schoolbook (its cost is d^2 word products instead of d^2 N^2 / 64^2).
 * q must be odd and below 2^61, so that 32 products of residues fit in 128 bits.
 */
static uint64_t reduce_coeff(const uint64_t *mag, int32_t w, int neg, uint64_t q)
{
    u128 r = 0;
    for (int32_t k = w - 1; k >= 0; --k) r = ((r << 64) | mag[k]) % q;
    uint64_t v = (uint64_t)r;
    return (neg && v) ? q - v : v;
}

int oracle_polymul_mod(const uint64_t *a, int64_t da, int32_t Na,
                       const uint64_t *b, int64_t db, int32_t Nb,
                       uint64_t q, uint64_t *c, int nthreads)
{
    if (da < 0 || db < 0 || Na < 1 || Nb < 1 || q < 3 || !(q & 1) || (q >> 61)) return -1;
    if (da == 0 || db == 0) return 0;
    int32_t wa = (Na + 63) / 64, wb = (Nb + 63) / 64;
    int64_t nout = da + db - 1;
    uint64_t *amag, *bmag;
    unsigned char *aneg, *bneg;
    if (prepare(a, da, Na, wa, &amag, &aneg) || prepare(b, db, Nb, wb, &bmag, &bneg)) return -1;
    uint64_t *ar = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)da);
    uint64_t *br = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)db);
    if (!ar || !br) { free(ar); free(br); free(amag); free(aneg); free(bmag); free(bneg); return -1; }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (int64_t l = 0; l < da; ++l) ar[l] = reduce_coeff(amag + (size_t)l * wa, wa, aneg[l], q);
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int64_t m = 0; m < db; ++m) br[m] = reduce_coeff(bmag + (size_t)m * wb, wb, bneg[m], q);
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < nout; ++i) {
        int64_t lo = i - (db - 1) > 0 ? i - (db - 1) : 0;
        int64_t hi = i < da - 1 ? i : da - 1;
        u128 acc = 0;
        int n = 0;
        for (int64_t l = lo; l <= hi; ++l) {
            acc += (u128)ar[l] * br[i - l];      /* each product is below 2^122 */
            if (++n == 32) { acc %= q; n = 0; }
        }
        c[i] = (uint64_t)(acc % q);
    }
    free(ar); free(br); free(amag); free(aneg); free(bmag); free(bneg);
    return 0;
}

/* Number of threads an OpenMP region actually gets with the given request. */
int oracle_threads(int nthreads)
{
    int n = 1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
    {
#pragma omp single
        n = omp_get_num_threads();
    }
#endif
    return n;
}
