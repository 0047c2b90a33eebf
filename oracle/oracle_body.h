/*
 * Body of the CPU oracle, included twice by stencil_oracle.c: once with
 * REAL = double (the reference arithmetic) and once with REAL = float (the
 * single-precision storage-and-compute form evaluated in the same order).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this file.
 *
 * Every update below is the per-point expression of the paper's listings,
 * written in the listing's left-to-right C order, so that each '*' and '+' is
 * one correctly rounded IEEE operation (the file is compiled with
 * -ffp-contract=off and without -ffast-math):
 *   7-point constant coefficient   : Listing 1 (Sec. I-A)
 *   7-point variable coefficient   : Listing 2 (Sec. I-A)
 *   25-point, radius 4, 13 weights : Listing 3 (Sec. I-A); the constant form
 *                                    holds each of the 13 weights fixed.
 * The time loop is the Jacobi-like two-array scheme of Sec. I: every sweep
 * reads only the previous level V and writes U, then the roles swap.
 */

/* Element (k, j, i) of a padded array; k, j, i are padded coordinates. */
#define AT(p, k, j, i) (p)[(long long)(k) * sz + (long long)(j) * sy + (long long)(i)]

static void SWEEP_NAME(int kind, int nx, int ny, int nz, int h,
                       long long sy, long long sz,
                       const REAL *V, REAL *U,
                       const REAL *c, const REAL *const *C, int nthreads)
{
    /* The listings loop k=1..N-2 (radius 1) and k=4..N-5 (radius 4) over an
     * array whose extent N includes the halo; here the interior is
     * [h, h+n) on every axis and the halo is at least the radius. */
    int k;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (k = h; k < h + nz; k++) {
        for (int j = h; j < h + ny; j++) {
            for (int i = h; i < h + nx; i++) {
                REAL u;
                if (kind == ORACLE_7C) {
                    /* Listing 1 */
                    u = c[0] * AT(V, k, j, i)
                      + c[1] * (AT(V, k, j, i + 1) + AT(V, k, j, i - 1))
                      + c[1] * (AT(V, k, j + 1, i) + AT(V, k, j - 1, i))
                      + c[1] * (AT(V, k + 1, j, i) + AT(V, k - 1, j, i));
                } else if (kind == ORACLE_7V) {
                    /* Listing 2: C1..C6 weight +x, -x, +y, -y, +z, -z */
                    u = AT(C[0], k, j, i) * AT(V, k, j, i)
                      + AT(C[1], k, j, i) * AT(V, k, j, i + 1)
                      + AT(C[2], k, j, i) * AT(V, k, j, i - 1)
                      + AT(C[3], k, j, i) * AT(V, k, j + 1, i)
                      + AT(C[4], k, j, i) * AT(V, k, j - 1, i)
                      + AT(C[5], k, j, i) * AT(V, k + 1, j, i)
                      + AT(C[6], k, j, i) * AT(V, k - 1, j, i);
                } else if (kind == ORACLE_25C) {
                    /* Listing 3 with every weight constant: c[0]=C00 and
                     * c[1..12]=C01..C12, radius-major, axis x, y, z. */
                    u = c[0] * AT(V, k, j, i)
                      + c[1] * (AT(V, k, j, i + 1) + AT(V, k, j, i - 1))
                      + c[2] * (AT(V, k, j + 1, i) + AT(V, k, j - 1, i))
                      + c[3] * (AT(V, k + 1, j, i) + AT(V, k - 1, j, i))
                      + c[4] * (AT(V, k, j, i + 2) + AT(V, k, j, i - 2))
                      + c[5] * (AT(V, k, j + 2, i) + AT(V, k, j - 2, i))
                      + c[6] * (AT(V, k + 2, j, i) + AT(V, k - 2, j, i))
                      + c[7] * (AT(V, k, j, i + 3) + AT(V, k, j, i - 3))
                      + c[8] * (AT(V, k, j + 3, i) + AT(V, k, j - 3, i))
                      + c[9] * (AT(V, k + 3, j, i) + AT(V, k - 3, j, i))
                      + c[10] * (AT(V, k, j, i + 4) + AT(V, k, j, i - 4))
                      + c[11] * (AT(V, k, j + 4, i) + AT(V, k, j - 4, i))
                      + c[12] * (AT(V, k + 4, j, i) + AT(V, k - 4, j, i));
                } else {
                    /* Listing 3 as printed: 13 coefficient arrays */
                    u = AT(C[0], k, j, i) * AT(V, k, j, i)
                      + AT(C[1], k, j, i) * (AT(V, k, j, i + 1) + AT(V, k, j, i - 1))
                      + AT(C[2], k, j, i) * (AT(V, k, j + 1, i) + AT(V, k, j - 1, i))
                      + AT(C[3], k, j, i) * (AT(V, k + 1, j, i) + AT(V, k - 1, j, i))
                      + AT(C[4], k, j, i) * (AT(V, k, j, i + 2) + AT(V, k, j, i - 2))
                      + AT(C[5], k, j, i) * (AT(V, k, j + 2, i) + AT(V, k, j - 2, i))
                      + AT(C[6], k, j, i) * (AT(V, k + 2, j, i) + AT(V, k - 2, j, i))
                      + AT(C[7], k, j, i) * (AT(V, k, j, i + 3) + AT(V, k, j, i - 3))
                      + AT(C[8], k, j, i) * (AT(V, k, j + 3, i) + AT(V, k, j - 3, i))
                      + AT(C[9], k, j, i) * (AT(V, k + 3, j, i) + AT(V, k - 3, j, i))
                      + AT(C[10], k, j, i) * (AT(V, k, j, i + 4) + AT(V, k, j, i - 4))
                      + AT(C[11], k, j, i) * (AT(V, k, j + 4, i) + AT(V, k, j - 4, i))
                      + AT(C[12], k, j, i) * (AT(V, k + 4, j, i) + AT(V, k - 4, j, i));
                }
                AT(U, k, j, i) = u;
            }
        }
    }
}

/* T sweeps of the two-array scheme.  buf0 holds u_0 on entry; buf1 must
 * carry the same halo (its interior is overwritten).  Level t ends up in
 * buffer t % 2, so on return u_T is in buffer (T % 2) and u_{T-1} in the
 * other one.  Returns T % 2, or -1 on invalid arguments. */
int RUN_NAME(int kind, int nx, int ny, int nz, int halo,
             long long sy, long long sz, REAL *buf0, REAL *buf1,
             const REAL *c, const REAL *const *C, int T, int nthreads)
{
    int radius = (kind == ORACLE_7C || kind == ORACLE_7V) ? 1 : 4;
    if (kind < 0 || kind > 3 || nx < 0 || ny < 0 || nz < 0 || halo < radius
        || T < 0 || !buf0 || !buf1 || nthreads < 1)
        return -1;
    if (sy < nx + 2LL * halo || sz < sy * (ny + 2LL * halo))
        return -1;
    if ((kind == ORACLE_7C || kind == ORACLE_25C) && !c)
        return -1;
    if ((kind == ORACLE_7V || kind == ORACLE_25V) && !C)
        return -1;
    for (int t = 0; t < T; t++) {
        const REAL *V = (t % 2 == 0) ? buf0 : buf1;
        REAL *U = (t % 2 == 0) ? buf1 : buf0;
        SWEEP_NAME(kind, nx, ny, nz, halo, sy, sz, V, U, c, C, nthreads);
    }
    return T % 2;
}

#undef AT
