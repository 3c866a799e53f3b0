/*
 * Plain CPU oracle in C -- TEST INFRASTRUCTURE ONLY.
 *
 * Only tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py
 * may load this library.  It shares no code, header, table or helper with the
 * HIP library: it is written independently from the paper so that the two can
 * be compared.
 *
 * What it computes (arXiv 2502.12428):
 *   oracle_fpow     g = f^k mod p                          (Algorithm 3, first line)
 *   oracle_delta1   Delta_1(g) = (g~^p - sum_t t^p)/p mod p (Algorithm 1, Prop. "delta1 formula")
 *   oracle_theta    u(Delta * a) mod p                      (Algorithm 2 applied to Delta*a; Section 3.4)
 *   oracle_height   the height loop with bound b            (Algorithm 3)
 *
 * Reading taken for Algorithm 1: the power g~^p is formed in Z/p^2 instead of
 * Z.  Every coefficient X of g~^p satisfies X = t^p (mod p) where t^p is the
 * subtracted term (or 0), so (X - t^p)/p mod p depends only on X mod p^2.  The
 * Python-integer tier (literal.py) computes over Z and pins this tier.
 *
 * Layout: a homogeneous polynomial of degree n in x1..x4 is held
 * dehomogenised (x4 dropped, Section 5.1 "Kronecker substitution") in a dense
 * cube: the coefficient of x1^a x2^b x3^c x4^(n-a-b-c) sits at
 * cube[(a*(n+1) + b)*(n+1) + c].  Entries with a+b+c > n are unused (zero).
 * Coefficient arrays at the interface are in B_n order: descending
 * lexicographic order of (e1,e2,e3,e4), enumerated below by nested loops
 * e1 = n..0, e2 = n-e1..0, e3 = n-e1-e2..0.
 *
 * Return codes: 0 ok, -1 bad argument, -2 arithmetic check failed (a
 * coefficient of g~^p - sum t^p not divisible by p), -3 out of memory.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_EINVAL (-1)
#define OR_EARITH (-2)
#define OR_ENOMEM (-3)

static size_t cube_len(int n) { size_t s = (size_t)n + 1; return s * s * s; }
static size_t cidx(int n, int a, int b, int c)
{
    size_t s = (size_t)n + 1;
    return ((size_t)a * s + (size_t)b) * s + (size_t)c;
}

/* Number of monomials of degree d in 4 variables, by counting. */
int64_t oracle_num_monomials(int d)
{
    if (d < 0) return 0;
    int64_t count = 0;
    for (int e1 = d; e1 >= 0; e1--)
        for (int e2 = d - e1; e2 >= 0; e2--)
            for (int e3 = d - e1 - e2; e3 >= 0; e3--)
                count++;
    return count;
}

/* Exponent tuples of B_d in descending lex order: exps[4*i + j]. */
int oracle_basis(int d, int32_t *exps)
{
    if (d < 0 || !exps) return OR_EINVAL;
    int64_t i = 0;
    for (int e1 = d; e1 >= 0; e1--)
        for (int e2 = d - e1; e2 >= 0; e2--)
            for (int e3 = d - e1 - e2; e3 >= 0; e3--) {
                exps[4 * i + 0] = e1;
                exps[4 * i + 1] = e2;
                exps[4 * i + 2] = e3;
                exps[4 * i + 3] = d - e1 - e2 - e3;
                i++;
            }
    return 0;
}

/* B_n-ordered array -> cube (values copied as they are). */
static void dense_to_cube(int n, const uint8_t *v, int32_t *cube)
{
    size_t i = 0;
    for (int e1 = n; e1 >= 0; e1--)
        for (int e2 = n - e1; e2 >= 0; e2--)
            for (int e3 = n - e1 - e2; e3 >= 0; e3--)
                cube[cidx(n, e1, e2, e3)] = v[i++];
}

/* cube -> B_n-ordered array. */
static void cube_to_dense(int n, const int32_t *cube, uint8_t *v)
{
    size_t i = 0;
    for (int e1 = n; e1 >= 0; e1--)
        for (int e2 = n - e1; e2 >= 0; e2--)
            for (int e3 = n - e1 - e2; e3 >= 0; e3--)
                v[i++] = (uint8_t)cube[cidx(n, e1, e2, e3)];
}

/*
 * C = A * B (schoolbook: every pair of terms), C of degree na+nb, zeroed here.
 * For each row (a1,a2) of A and each nonzero term b of B, the row of A is
 * added, scaled by b, into the row of C shifted by b.
 */
static void cube_mul(const int32_t *A, int na, const int32_t *B, int nb, int32_t *C)
{
    int nc = na + nb;
    memset(C, 0, cube_len(nc) * sizeof(int32_t));
    for (int a1 = 0; a1 <= na; a1++)
        for (int a2 = 0; a2 <= na - a1; a2++) {
            const int32_t *arow = A + cidx(na, a1, a2, 0);
            int alen = na - a1 - a2 + 1;
            for (int b1 = 0; b1 <= nb; b1++)
                for (int b2 = 0; b2 <= nb - b1; b2++)
                    for (int b3 = 0; b3 <= nb - b1 - b2; b3++) {
                        int32_t bv = B[cidx(nb, b1, b2, b3)];
                        if (!bv) continue;
                        int32_t *crow = C + cidx(nc, a1 + b1, a2 + b2, b3);
                        for (int a3 = 0; a3 < alen; a3++)
                            crow[a3] += bv * arow[a3];
                    }
        }
}

static void cube_reduce(int32_t *C, int n, int32_t m)
{
    size_t len = cube_len(n);
    for (size_t i = 0; i < len; i++) {
        int32_t r = C[i] % m;
        C[i] = r < 0 ? r + m : r;
    }
}

static int valid_prime(int p)
{
    if (p < 2 || p > 97) return 0;
    for (int q = 2; q * q <= p; q++)
        if (p % q == 0) return 0;
    return 1;
}

/* out = f^k mod p, f of degree 4 (35 coefficients in B_4 order), out in B_{4k} order. */
int oracle_fpow(int p, int k, const uint8_t *f, uint8_t *out)
{
    if (!valid_prime(p) || k < 0 || !f || !out) return OR_EINVAL;
    for (int i = 0; i < 35; i++)
        if (f[i] >= p) return OR_EINVAL;
    int nmax = 4 * k;
    int32_t *F = calloc(cube_len(4), sizeof(int32_t));
    int32_t *A = calloc(cube_len(nmax), sizeof(int32_t));
    int32_t *C = calloc(cube_len(nmax), sizeof(int32_t));
    if (!F || !A || !C) { free(F); free(A); free(C); return OR_ENOMEM; }
    dense_to_cube(4, f, F);
    A[0] = 1; /* the constant 1, degree 0 */
    for (int j = 0; j < k; j++) {
        cube_mul(A, 4 * j, F, 4, C);
        cube_reduce(C, 4 * (j + 1), p);
        int32_t *t = A; A = C; C = t;
    }
    cube_to_dense(nmax, A, out);
    free(F); free(A); free(C);
    return 0;
}

static int32_t powmod(int32_t b, int e, int32_t m)
{
    int64_t r = 1 % m;
    for (int i = 0; i < e; i++) r = (r * b) % m;
    return (int32_t)r;
}

/*
 * delta_out = Delta_1(g) for g homogeneous of degree d with coefficients in
 * [0,p) given in B_d order; delta_out in B_{pd} order.  Algorithm 1:
 *   D <- g~^p ; D <- D - t^p for every term t ; D <- D / p ; reduce mod p.
 */
int oracle_delta1(int p, int d, const uint8_t *g, uint8_t *delta_out)
{
    if (!valid_prime(p) || d < 0 || !g || !delta_out) return OR_EINVAL;
    int64_t lg = oracle_num_monomials(d);
    for (int64_t i = 0; i < lg; i++)
        if (g[i] >= p) return OR_EINVAL;
    int32_t p2 = p * p;
    int nD = p * d;
    int32_t *G = calloc(cube_len(d), sizeof(int32_t));
    int32_t *A = calloc(cube_len(nD), sizeof(int32_t));
    int32_t *C = calloc(cube_len(nD), sizeof(int32_t));
    if (!G || !A || !C) { free(G); free(A); free(C); return OR_ENOMEM; }
    dense_to_cube(d, g, G);                      /* the lift g~, coefficients in [0,p) */
    memcpy(A, G, cube_len(d) * sizeof(int32_t)); /* g~^1 */
    for (int k = 1; k < p; k++) {                /* g~^(k+1) = g~^k * g~ in Z/p^2 */
        cube_mul(A, k * d, G, d, C);
        cube_reduce(C, (k + 1) * d, p2);
        int32_t *t = A; A = C; C = t;
    }
    /* subtract t^p = b^p x^(pJ) for every term b x^J of g~ */
    for (int e1 = 0; e1 <= d; e1++)
        for (int e2 = 0; e2 <= d - e1; e2++)
            for (int e3 = 0; e3 <= d - e1 - e2; e3++) {
                int32_t b = G[cidx(d, e1, e2, e3)];
                if (!b) continue;
                size_t at = cidx(nD, p * e1, p * e2, p * e3);
                int32_t v = (A[at] - powmod(b, p, p2)) % p2;
                A[at] = v < 0 ? v + p2 : v;
            }
    /* every coefficient must now be divisible by p; divide */
    int rc = 0;
    for (int e1 = 0; e1 <= nD && !rc; e1++)
        for (int e2 = 0; e2 <= nD - e1 && !rc; e2++)
            for (int e3 = 0; e3 <= nD - e1 - e2; e3++) {
                int32_t v = A[cidx(nD, e1, e2, e3)];
                if (v % p) { rc = OR_EARITH; break; }
                A[cidx(nD, e1, e2, e3)] = v / p;
            }
    if (!rc) cube_to_dense(nD, A, delta_out);
    free(G); free(A); free(C);
    return rc;
}

/*
 * out = u(Delta * a) mod p for a of degree d = 4(p-1) and Delta of degree
 * D = p*d, both in B order.  A term Delta_delta x^delta times a_c x^c survives
 * u only when delta + c = (p-1,...,p-1) mod p (Algorithm 2); it then lands on
 * r = (delta + c - (p-1)1)/p, which has degree d.  So for each output r and
 * each input c the one contributing Delta term is delta = p*r + (p-1)1 - c,
 * present when all four of its exponents are >= 0.
 */
int oracle_theta(int p, const uint8_t *delta, const uint8_t *a, uint8_t *out)
{
    if (!valid_prime(p) || !delta || !a || !out) return OR_EINVAL;
    int d = 4 * (p - 1), nD = p * d;
    int64_t ld = oracle_num_monomials(d), lD = oracle_num_monomials(nD);
    for (int64_t i = 0; i < ld; i++) if (a[i] >= p) return OR_EINVAL;
    for (int64_t i = 0; i < lD; i++) if (delta[i] >= p) return OR_EINVAL;
    int32_t *Dc = calloc(cube_len(nD), sizeof(int32_t));
    int32_t *ex = malloc(sizeof(int32_t) * 4 * (size_t)ld);
    if (!Dc || !ex) { free(Dc); free(ex); return OR_ENOMEM; }
    dense_to_cube(nD, delta, Dc);
    oracle_basis(d, ex);
    for (int64_t r = 0; r < ld; r++) {
        int64_t acc = 0;
        for (int64_t c = 0; c < ld; c++) {
            if (!a[c]) continue;
            int dl[4], ok = 1;
            for (int j = 0; j < 4; j++) {
                dl[j] = p * ex[4 * r + j] + (p - 1) - ex[4 * c + j];
                if (dl[j] < 0) ok = 0;
            }
            if (!ok) continue;
            acc += (int64_t)Dc[cidx(nD, dl[0], dl[1], dl[2])] * a[c];
        }
        out[r] = (uint8_t)(acc % p);
    }
    free(Dc); free(ex);
    return 0;
}

/* g not in m^[p]: some nonzero term has every exponent < p. */
static int outside_frobenius_power(int p, int d, const uint8_t *g, const int32_t *ex, int64_t ld)
{
    (void)d;
    for (int64_t i = 0; i < ld; i++) {
        if (!g[i]) continue;
        if (ex[4 * i] < p && ex[4 * i + 1] < p && ex[4 * i + 2] < p && ex[4 * i + 3] < p)
            return 1;
    }
    return 0;
}

/*
 * Algorithm 3 for a quartic f (35 coefficients in B_4 order, values in [0,p)).
 * Returns the height 1..bound, 0 for infinity (no height <= bound), or a
 * negative error code.  If theta_iters is not NULL it receives the number of
 * times theta was applied.
 */
int oracle_height(int p, const uint8_t *f, int bound, int *theta_iters)
{
    if (!valid_prime(p) || !f || bound < 1) return OR_EINVAL;
    int d = 4 * (p - 1), nD = p * d;
    int64_t ld = oracle_num_monomials(d), lD = oracle_num_monomials(nD);
    uint8_t *g = malloc((size_t)ld), *g2 = malloc((size_t)ld), *Dl = malloc((size_t)lD);
    int32_t *ex = malloc(sizeof(int32_t) * 4 * (size_t)ld);
    int rc;
    if (theta_iters) *theta_iters = 0;
    if (!g || !g2 || !Dl || !ex) { rc = OR_ENOMEM; goto done; }
    oracle_basis(d, ex);
    rc = oracle_fpow(p, p - 1, f, g);
    if (rc) goto done;
    if (outside_frobenius_power(p, d, g, ex, ld)) { rc = 1; goto done; }
    rc = oracle_delta1(p, d, g, Dl);
    if (rc) goto done;
    for (int h = 2;; h++) {
        if (bound < h) { rc = 0; break; }
        rc = oracle_theta(p, Dl, g, g2);
        if (rc) break;
        if (theta_iters) (*theta_iters)++;
        uint8_t *t = g; g = g2; g2 = t;
        if (outside_frobenius_power(p, d, g, ex, ld)) { rc = h; break; }
    }
done:
    free(g); free(g2); free(Dl); free(ex);
    return rc;
}
