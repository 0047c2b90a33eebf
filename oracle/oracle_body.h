/*
 * Body of the CPU oracle, included twice by stencil_oracle.c: once with
 * REAL = double (the reference arithmetic) and once with REAL = float (the
 * single-precision storage-and-compute form evaluated in the same order).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this file.
 *
 * Every update below evaluates the per-point expression of the paper's
 * listings term by term, from tables of neighbour offsets, in the listing's
 * left-to-right C order, so that each '*' and '+' is one correctly rounded
 * IEEE operation (the file is compiled with -ffp-contract=off and without
 * -ffast-math):
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
    /* Element stride of one step along x, y and z. */
    const long long axis_step[3] = {1, sy, sz};
    /* Neighbour of each radius-1 variable weight C1..C6: +x, -x, +y, -y, +z, -z. */
    const long long nb7[6] = {1, -1, sy, -sy, sz, -sz};
    /* The listings loop k=1..N-2 (radius 1) and k=4..N-5 (radius 4) over an
     * array whose extent N includes the halo; here the interior is
     * [h, h+n) on every axis and the halo is at least the radius. */
    int k;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (k = h; k < h + nz; k++) {
        for (int j = h; j < h + ny; j++) {
            for (int i = h; i < h + nx; i++) {
                const long long o = (long long)k * sz + (long long)j * sy + i;
                const REAL *v = V + o;   /* v[d]: the neighbour at element offset d */
                REAL u;
                if (kind == ORACLE_7C) {
                    /* Listing 1: c0 at the centre, then c1 on the neighbour
                     * pair of each axis x, y, z, + side first */
                    u = c[0] * v[0];
                    for (int a = 0; a < 3; a++)
                        u = u + c[1] * (v[axis_step[a]] + v[-axis_step[a]]);
                } else if (kind == ORACLE_7V) {
                    /* Listing 2: array C0 at the centre, C1..C6 each on one
                     * neighbour, in the order of nb7 */
                    u = C[0][o] * v[0];
                    for (int m = 1; m <= 6; m++)
                        u = u + C[m][o] * v[nb7[m - 1]];
                } else {
                    /* Listing 3: weight 0 at the centre, then weight
                     * 3(r-1)+a+1 on the pair at distance r along axis a,
                     * radius-major and axis x, y, z inner, + side first; the
                     * constant form holds each of the 13 weights fixed */
                    u = (kind == ORACLE_25C ? c[0] : C[0][o]) * v[0];
                    for (int r = 1; r <= 4; r++) {
                        for (int a = 0; a < 3; a++) {
                            const int q = 3 * (r - 1) + a + 1;
                            const REAL w = kind == ORACLE_25C ? c[q] : C[q][o];
                            u = u + w * (v[r * axis_step[a]] + v[-r * axis_step[a]]);
                        }
                    }
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
