/*
 * Oracle: the HISQ staggered stencil D, written out from its definition.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code with
 * the GPU library.
 *
 * The paper writes the quark matrix as M = D + 2m with D the anti-Hermitian HISQ
 * matrix (section 2, the text around Eq. (1)).  D is a fat-link one-hop term
 * plus a Naik (long-link) three-hop term; the staggered phases, the coefficients
 * and the antiperiodic time boundary sign are already folded into the links F
 * and L that this file receives:
 *
 *   (D psi)(x) = sum_mu [  F_mu(x) psi(x+mu)      - F_mu(x-mu)^H psi(x-mu)
 *                        + L_mu(x) psi(x+3mu)     - L_mu(x-3mu)^H psi(x-3mu) ]
 *
 * with every coordinate taken modulo the lattice extent.  No factor 1/2 (MILC
 * normalisation, fixed by the free-field spectrum against the lambda_max ~ 23
 * quoted in section 2).
 *
 * Layout (canonical, x fastest): dims = {X, Y, Z, T};
 *   links  [4][T][Z][Y][X][3][3] complex double, row-major colour matrix
 *   fields [T][Z][Y][X][3]       complex double
 * Plain loops, one output site at a time; OpenMP over sites.
 */
#include <complex.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

static int64_t lex_of(const int d[4], const int x[4]) {
    return (((int64_t)x[3] * d[2] + x[2]) * d[1] + x[1]) * d[0] + x[0];
}

static void coords_of(const int d[4], int64_t lex, int x[4]) {
    for (int mu = 0; mu < 4; ++mu) {
        x[mu] = (int)(lex % d[mu]);
        lex /= d[mu];
    }
}

static int wrap(int v, int n) {
    int r = v % n;
    return r < 0 ? r + n : r;
}

/* acc += U v */
static void mul_add(const cplx *U, const cplx *v, cplx *acc) {
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) acc[a] += U[3 * a + b] * v[b];
}

/* acc -= U^H v */
static void adj_mul_sub(const cplx *U, const cplx *v, cplx *acc) {
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) acc[a] -= conj(U[3 * b + a]) * v[b];
}

/* (D psi)(x) at the one site with lexicographic index lex. */
void oracle_dslash_site(const int d[4], const cplx *F, const cplx *L, const cplx *in,
                        int64_t lex, cplx *out3) {
    const int64_t V = (int64_t)d[0] * d[1] * d[2] * d[3];
    int x[4];
    coords_of(d, lex, x);
    cplx acc[3] = {0, 0, 0};
    for (int mu = 0; mu < 4; ++mu) {
        const cplx *links[2] = {F + (int64_t)mu * V * 9, L + (int64_t)mu * V * 9};
        const int hops[2] = {1, 3};
        for (int h = 0; h < 2; ++h) {
            int xf[4], xb[4];
            memcpy(xf, x, sizeof xf);
            memcpy(xb, x, sizeof xb);
            xf[mu] = wrap(x[mu] + hops[h], d[mu]);
            xb[mu] = wrap(x[mu] - hops[h], d[mu]);
            const int64_t lf = lex_of(d, xf), lb = lex_of(d, xb);
            mul_add(links[h] + lex * 9, in + lf * 3, acc);      /* forward hop  */
            adj_mul_sub(links[h] + lb * 9, in + lb * 3, acc);   /* backward hop */
        }
    }
    out3[0] = acc[0];
    out3[1] = acc[1];
    out3[2] = acc[2];
}

/*
 * out = D in on the rows selected by `rows`: 0 = even sites only, 1 = odd sites
 * only, 2 = every site.  Rows that are not computed are set to zero.  Site
 * parity is (x+y+z+t) mod 2.
 */
void oracle_dslash(const int d[4], const cplx *F, const cplx *L, const cplx *in,
                   cplx *out, int rows, int nthreads) {
    const int64_t V = (int64_t)d[0] * d[1] * d[2] * d[3];
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        int x[4];
        coords_of(d, s, x);
        const int par = (x[0] + x[1] + x[2] + x[3]) & 1;
        if (rows == 2 || rows == par) {
            oracle_dslash_site(d, F, L, in, s, out + s * 3);
        } else {
            out[s * 3 + 0] = 0;
            out[s * 3 + 1] = 0;
            out[s * 3 + 2] = 0;
        }
    }
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
