/*
 * FP64 CPU oracle for the FFT translational BPMF scan.
 *
 * TEST INFRASTRUCTURE ONLY.  Tests, the smoke check and the benchmark's CPU
 * baseline call it; the product library never does, and the two share no
 * code, headers or tables.  It is deliberately plain and slow: every result
 * is the definition written out in double precision, with no FFT.
 *
 * What is computed (Nguyen, Zhou & Minh, "Using the Fast Fourier Transform
 * in Binding Free Energy Calculations"):
 *   - receptor grids, Eq. 7 with the three pair terms of Eqs. 4-6 and the
 *     short-range exclusion of the FFT-based BPMF estimation section;
 *   - receptor/ligand occupancy grids, Eq. 10 (radius scaled by occ_f);
 *   - ligand placement: random rotation about the centroid ("Ligand
 *     Sampling"), lowest coordinates two spacings from the i=0, j=0, k=0
 *     planes, box = coordinates plus two spacings;
 *   - the interaction energy of Eq. 8 at every box-valid translation,
 *     evaluated directly: each ligand atom's weight is spread with trilinear
 *     (8-point) weights, so the correlation equals the trilinear
 *     interpolation of the receptor grid at the atom position;
 *   - the steric-clash test of Eq. 10 (exact integer arithmetic);
 *   - per-configuration partial sums of the sample mean of Eq. 2.
 *
 * Readings where the paper is silent (kept identical in the GPU library):
 *   - spreading is trilinear, not the ten-point scheme of Qin & Zhou;
 *   - the ligand sits at u_i + t (translation t applied to the ligand);
 *   - placed coordinates are rounded to a 2^-16 grid-unit lattice, so box
 *     extents and occupancy membership are exact integer decisions;
 *   - occupancy membership: |n - u_i| < rho_i  <=>  D < ceil(rho_i^2 2^32)
 *     with D = |2^16 n - U_i|^2 an integer;
 *   - grid indices are taken modulo the FFT edge n_fft over the zero-padded
 *     receptor grid (the periodic convention of the FFT).
 *
 * Parity status of each function is pinned by the CPU tests (brute force,
 * closed forms, the correlation theorem via numpy.fft); see the tests.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define LAT 65536.0 /* placement lattice: 2^16 points per grid unit */

static inline long long imod(long long a, long long n) {
    if (a >= 0 && a < n) return a;
    long long r = a % n;
    return r < 0 ? r + n : r;
}

/* ---------------------------------------------------------------------- */
/* Eq. 7 receptor grids.                                                   */
/*   ch 0  ELE : 332.05 * sum_j q_j / r                      (Eq. 4)       */
/*   ch 1  LJr : sum_j sqrt(eps_j) sigma_j^6 / r^12          (Eq. 5)       */
/*   ch 2  LJa : sum_j sqrt(eps_j) sigma_j^3 / r^6           (Eq. 6, the   */
/*               ligand weight carries the factor -2)                      */
/* mode 0 (occupancy): V = 0 for r < 2^-1/6 sigma_j on all three channels. */
/* mode 1 (cap): V = 0 for r < 2^-1/6 sigma_j on ELE and LJa only; LJr is  */
/*               kept and the grid value is clamped to `cap`.              */
/* occ (if non-NULL): Eq. 10 with radius occ_f * 2^-1/6 sigma_j.           */
/* Grid point (x,y,z) sits at origin + h*(x,y,z); layout [z][y][x].        */
/* ---------------------------------------------------------------------- */
void orc_receptor_grids(int n_atoms, const double *xyz, const double *q,
                        const double *sigma, const double *eps, int n_rec,
                        double h, const double *origin, int mode, double cap,
                        double occ_f, double *grids, uint8_t *occ) {
    const double two_m16 = pow(2.0, -1.0 / 6.0);
    const long long n3 = (long long)n_rec * n_rec * n_rec;
#pragma omp parallel for schedule(dynamic, 1)
    for (int z = 0; z < n_rec; ++z) {
        for (int y = 0; y < n_rec; ++y) {
            for (int x = 0; x < n_rec; ++x) {
                double px = origin[0] + h * x, py = origin[1] + h * y, pz = origin[2] + h * z;
                double ele = 0.0, ljr = 0.0, lja = 0.0;
                int hit = 0;
                for (int j = 0; j < n_atoms; ++j) {
                    double dx = xyz[3 * j] - px, dy = xyz[3 * j + 1] - py, dz = xyz[3 * j + 2] - pz;
                    double r = sqrt(dx * dx + dy * dy + dz * dz);
                    double rex = two_m16 * sigma[j];
                    if (r < occ_f * rex) hit = 1;
                    double s3 = sigma[j] * sigma[j] * sigma[j];
                    double se = sqrt(eps[j]);
                    double r6 = r * r * r * r * r * r;
                    if (r >= rex) {
                        ele += 332.05 * q[j] / r;
                        lja += se * s3 / r6;
                        ljr += se * s3 * s3 / (r6 * r6);
                    } else if (mode == 1) {
                        ljr += se * s3 * s3 / (r6 * r6);
                    }
                }
                if (mode == 1 && ljr > cap) ljr = cap;
                long long idx = ((long long)z * n_rec + y) * n_rec + x;
                grids[idx] = ele;
                grids[n3 + idx] = ljr;
                grids[2 * n3 + idx] = lja;
                if (occ) occ[idx] = (uint8_t)hit;
            }
        }
    }
}

/* Ligand weights gamma_i per channel (Eqs. 4-6): q, sqrt(eps) sigma^6,
 * -2 sqrt(eps) sigma^3.  Layout [n_atoms][3]. */
void orc_ligand_weights(int n, const double *q, const double *sigma, const double *eps,
                        double *gamma) {
    for (int i = 0; i < n; ++i) {
        double s3 = sigma[i] * sigma[i] * sigma[i];
        double se = sqrt(eps[i]);
        gamma[3 * i + 0] = q[i];
        gamma[3 * i + 1] = se * s3 * s3;
        gamma[3 * i + 2] = -2.0 * se * s3;
    }
}

/* Occupancy membership threshold in lattice units: ceil(rho^2 2^32) with
 * rho = occ_f 2^-1/6 sigma / h (grid units). */
double orc_occ_threshold(double sigma, double occ_f, double h) {
    double rho = occ_f * pow(2.0, -1.0 / 6.0) * sigma / h;
    return ceil(rho * rho * 4294967296.0);
}

/* Placement of one configuration ("Ligand Sampling" and the placement rule
 * of the FFT-based BPMF estimation section).
 *   centroid c = mean_i X_i (unweighted)
 *   Y_i = R(q) (X_i - c), R from the normalised quaternion (w,x,y,z)
 *   u_i = (Y_i - min_k Y_k) / h + 2, rounded to the 2^-16 lattice
 *   box_d = ceil(max_i u_i,d) + 2
 * Returns 0, or -1 for a zero quaternion. */
int orc_place(int n, const double *xyz, const double *quat, double h, double *u, int *box) {
    double nq = sqrt(quat[0] * quat[0] + quat[1] * quat[1] + quat[2] * quat[2] + quat[3] * quat[3]);
    if (!(nq > 0.0)) return -1;
    double w = quat[0] / nq, x = quat[1] / nq, y = quat[2] / nq, z = quat[3] / nq;
    double R[3][3] = {
        {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y)},
        {2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x)},
        {2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)}};
    double c[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) c[d] += xyz[3 * i + d];
    for (int d = 0; d < 3; ++d) c[d] /= n;
    double mn[3] = {INFINITY, INFINITY, INFINITY};
    for (int i = 0; i < n; ++i) {
        double v[3] = {xyz[3 * i] - c[0], xyz[3 * i + 1] - c[1], xyz[3 * i + 2] - c[2]};
        for (int d = 0; d < 3; ++d) {
            u[3 * i + d] = R[d][0] * v[0] + R[d][1] * v[1] + R[d][2] * v[2];
            if (u[3 * i + d] < mn[d]) mn[d] = u[3 * i + d];
        }
    }
    double mx[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            double v = (u[3 * i + d] - mn[d]) / h + 2.0;
            v = round(v * LAT) / LAT;
            u[3 * i + d] = v;
            if (v > mx[d]) mx[d] = v;
        }
    for (int d = 0; d < 3; ++d) box[d] = (int)ceil(mx[d]) + 2;
    return 0;
}

/* Value of receptor grid channel array g (n_rec^3) at integer index c,
 * taken modulo n_fft over the zero-padded grid. */
static inline double gval(const double *g, int n_rec, int n_fft, long long cx, long long cy,
                          long long cz) {
    cx = imod(cx, n_fft);
    cy = imod(cy, n_fft);
    cz = imod(cz, n_fft);
    if (cx >= n_rec || cy >= n_rec || cz >= n_rec) return 0.0;
    return g[(cz * n_rec + cy) * n_rec + cx];
}

/* Interaction energy (Eq. 8 with the ligand translated by t) at every
 * box-valid translation t, written to psi[tz][ty][tx], t_d < n_rec - box_d:
 *   Psi(t) = sum_i sum_ch gamma_i,ch sum_{delta in {0,1}^3}
 *            w_delta(u_i) G_ch(floor(u_i) + t + delta)
 * with trilinear weights w_delta = prod_d (delta_d ? f_d : 1 - f_d).
 * If mask is non-NULL, translations with mask != 0 are skipped (left 0). */
void orc_direct_energy(int n_rec, int n_fft, const double *grids, int n_atoms,
                       const double *u, const double *gamma, const int *box,
                       const uint8_t *mask, double *psi) {
    const long long n3 = (long long)n_rec * n_rec * n_rec;
    int V[3];
    for (int d = 0; d < 3; ++d) V[d] = n_rec - box[d];
    if (V[0] <= 0 || V[1] <= 0 || V[2] <= 0) return;
    for (int tz = 0; tz < V[2]; ++tz)
        for (int ty = 0; ty < V[1]; ++ty)
            for (int tx = 0; tx < V[0]; ++tx) {
                long long lin = ((long long)tz * V[1] + ty) * V[0] + tx;
                if (mask && mask[lin]) {
                    psi[lin] = 0.0;
                    continue;
                }
                double acc = 0.0;
                for (int i = 0; i < n_atoms; ++i) {
                    double fl[3], fr[3];
                    long long a[3];
                    for (int d = 0; d < 3; ++d) {
                        a[d] = (long long)floor(u[3 * i + d]);
                        fr[d] = u[3 * i + d] - (double)a[d];
                        fl[d] = 1.0 - fr[d];
                    }
                    for (int ch = 0; ch < 3; ++ch) {
                        const double *g = grids + ch * n3;
                        double s = 0.0;
                        for (int dz = 0; dz < 2; ++dz)
                            for (int dy = 0; dy < 2; ++dy)
                                for (int dx = 0; dx < 2; ++dx) {
                                    double w = (dx ? fr[0] : fl[0]) * (dy ? fr[1] : fl[1]) *
                                               (dz ? fr[2] : fl[2]);
                                    s += w * gval(g, n_rec, n_fft, a[0] + tx + dx,
                                                  a[1] + ty + dy, a[2] + tz + dz);
                                }
                        acc += gamma[3 * i + ch] * s;
                    }
                }
                psi[lin] = acc;
            }
}

/* Ligand occupancy points (Eq. 10): all integer n with
 * |2^16 n - U_i|^2 < thr_i for some atom i, listed once each.
 * Returns the number of points; pts has room for cap*3 ints. */
static int occ_points(int n_atoms, const double *u, const double *thr, int *pts, int cap) {
    /* bounding cube of all balls */
    long long lo[3], hi[3];
    for (int d = 0; d < 3; ++d) { lo[d] = 1LL << 40; hi[d] = -(1LL << 40); }
    for (int i = 0; i < n_atoms; ++i) {
        double r = sqrt(thr[i]) / LAT + 1.0;
        for (int d = 0; d < 3; ++d) {
            long long a = (long long)floor(u[3 * i + d] - r), b = (long long)ceil(u[3 * i + d] + r);
            if (a < lo[d]) lo[d] = a;
            if (b > hi[d]) hi[d] = b;
        }
    }
    long long *U = (long long *)malloc(sizeof(long long) * 3 * (n_atoms > 0 ? n_atoms : 1));
    if (!U) return -1;
    for (int i = 0; i < 3 * n_atoms; ++i) U[i] = (long long)llround(u[i] * LAT);
    int np = 0;
    for (long long z = lo[2]; z <= hi[2]; ++z)
        for (long long y = lo[1]; y <= hi[1]; ++y)
            for (long long x = lo[0]; x <= hi[0]; ++x) {
                for (int i = 0; i < n_atoms; ++i) {
                    long long ex = x * 65536LL - U[3 * i], ey = y * 65536LL - U[3 * i + 1],
                              ez = z * 65536LL - U[3 * i + 2];
                    long long D = ex * ex + ey * ey + ez * ez;
                    if ((double)D < thr[i]) {
                        if (np < cap) {
                            pts[3 * np] = (int)x;
                            pts[3 * np + 1] = (int)y;
                            pts[3 * np + 2] = (int)z;
                        }
                        ++np;
                        break;
                    }
                }
            }
    free(U);
    return np;
}

static int cmp_key(const void *a, const void *b) {
    double ka = *(const double *)a, kb = *(const double *)b;
    return (ka > kb) - (ka < kb);
}

/* Steric clash (Eq. 10 and the text after it) at every box-valid t:
 * clash(t) = 1 iff some ligand occupancy point n has O_R((n + t) mod n_fft)
 * = 1, with O_R zero outside the n_rec^3 receptor grid.
 * Returns the number of ligand occupancy points, or -1 on allocation failure. */
int orc_clash(int n_rec, int n_fft, const uint8_t *occ, int n_atoms, const double *u,
              const double *thr, const int *box, uint8_t *clash) {
    int V[3];
    for (int d = 0; d < 3; ++d) V[d] = n_rec - box[d];
    int cap = 1 << 16;
    int *pts = (int *)malloc(sizeof(int) * 3 * cap);
    if (!pts) return -1;
    int np = occ_points(n_atoms, u, thr, pts, cap);
    if (np < 0) {
        free(pts);
        return -1;
    }
    if (np > cap) {
        free(pts);
        cap = np;
        pts = (int *)malloc(sizeof(int) * 3 * cap);
        if (!pts) return -1;
        occ_points(n_atoms, u, thr, pts, cap);
    }
    /* Visit the points farthest from their mean first: only the order of the
     * search changes (it stops at the first hit), never the result. */
    double mc[3] = {0, 0, 0};
    for (int p = 0; p < np; ++p)
        for (int d = 0; d < 3; ++d) mc[d] += pts[3 * p + d];
    for (int d = 0; d < 3; ++d) mc[d] /= (np > 0 ? np : 1);
    struct kp { double key; int x, y, z; } *ord = (struct kp *)malloc(sizeof(struct kp) * (np > 0 ? np : 1));
    if (!ord) {
        free(pts);
        return -1;
    }
    for (int p = 0; p < np; ++p) {
        double dx = pts[3 * p] - mc[0], dy = pts[3 * p + 1] - mc[1], dz = pts[3 * p + 2] - mc[2];
        ord[p].key = -(dx * dx + dy * dy + dz * dz);
        ord[p].x = pts[3 * p];
        ord[p].y = pts[3 * p + 1];
        ord[p].z = pts[3 * p + 2];
    }
    qsort(ord, np, sizeof(struct kp), cmp_key);
    if (V[0] > 0 && V[1] > 0 && V[2] > 0) {
        for (int tz = 0; tz < V[2]; ++tz)
            for (int ty = 0; ty < V[1]; ++ty)
                for (int tx = 0; tx < V[0]; ++tx) {
                    long long lin = ((long long)tz * V[1] + ty) * V[0] + tx;
                    uint8_t c = 0;
                    for (int p = 0; p < np && !c; ++p) {
                        long long x = imod(ord[p].x + tx, n_fft);
                        long long y = imod(ord[p].y + ty, n_fft);
                        long long z = imod(ord[p].z + tz, n_fft);
                        if (x < n_rec && y < n_rec && z < n_rec &&
                            occ[(z * n_rec + y) * n_rec + x])
                            c = 1;
                    }
                    clash[lin] = c;
                }
    }
    free(ord);
    free(pts);
    return np;
}

/* Per-configuration partial of the sample mean of Eq. 2 over n samples:
 * out = {m, s, n_valid, n_finite, psi_min, argmin} with x = -beta Psi over
 * finite samples (clash -> +inf is excluded from the sum, counted in n):
 *   m = max x, s = sum exp(x - m), psi_min = min Psi, argmin = lowest index. */
void orc_partial(long long n, const double *psi, const uint8_t *clash, double beta,
                 double *out) {
    double m = -INFINITY, pmin = INFINITY;
    long long nf = 0, amin = -1;
    for (long long k = 0; k < n; ++k) {
        if (clash && clash[k]) continue;
        ++nf;
        double x = -beta * psi[k];
        if (x > m) m = x;
        if (psi[k] < pmin) { pmin = psi[k]; amin = k; }
    }
    double s = 0.0;
    if (nf > 0)
        for (long long k = 0; k < n; ++k) {
            if (clash && clash[k]) continue;
            s += exp(-beta * psi[k] - m);
        }
    out[0] = m;
    out[1] = s;
    out[2] = (double)n;
    out[3] = (double)nf;
    out[4] = pmin;
    out[5] = (double)amin;
}

/* Whole configuration set of one ligand against one receptor snapshot:
 * placement, clash test (if occ non-NULL), direct energies (only at clash-
 * free translations unless raw_everywhere), partial.  OpenMP over
 * configurations.  partials: [n_cfg][6] as orc_partial; box_out [n_cfg][3]
 * may be NULL.  Returns 0, or -1 on failure. */
int orc_scan(int n_rec, int n_fft, const double *grids, const uint8_t *occ, double h,
             int n_atoms, const double *conf_xyz, const double *gamma, const double *thr,
             int n_cfg, const int *cfg_conf, const double *cfg_quat, double beta,
             int raw_everywhere, double *partials, int *box_out) {
    int fail = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < n_cfg; ++c) {
        double *u = (double *)malloc(sizeof(double) * 3 * n_atoms);
        int box[3];
        if (!u || orc_place(n_atoms, conf_xyz + (size_t)cfg_conf[c] * 3 * n_atoms,
                            cfg_quat + 4 * c, h, u, box) != 0) {
            fail = 1;
            free(u);
            continue;
        }
        if (box_out) for (int d = 0; d < 3; ++d) box_out[3 * c + d] = box[d];
        long long V[3], nv = 1;
        for (int d = 0; d < 3; ++d) {
            V[d] = n_rec - box[d];
            if (V[d] < 0) V[d] = 0;
            nv *= V[d];
        }
        double *psi = (double *)calloc(nv > 0 ? nv : 1, sizeof(double));
        uint8_t *cl = occ ? (uint8_t *)calloc(nv > 0 ? nv : 1, 1) : NULL;
        if (!psi || (occ && !cl)) {
            fail = 1;
        } else if (nv > 0) {
            if (occ && orc_clash(n_rec, n_fft, occ, n_atoms, u, thr, box, cl) < 0) fail = 1;
            orc_direct_energy(n_rec, n_fft, grids, n_atoms, u, gamma, box,
                              raw_everywhere ? NULL : cl, psi);
        }
        orc_partial(nv, psi, cl, beta, partials + 6 * c);
        free(psi);
        free(cl);
        free(u);
    }
    return fail ? -1 : 0;
}

/* Dense ligand grid for one channel: trilinear spreading of weights w_i at
 * u_i onto an n_fft^3 periodic grid (the ligand grid G_L of Eq. 8). */
void orc_spread_dense(int n_fft, int n_atoms, const double *u, const double *w, double *out) {
    memset(out, 0, sizeof(double) * (size_t)n_fft * n_fft * n_fft);
    for (int i = 0; i < n_atoms; ++i) {
        long long a[3];
        double fr[3], fl[3];
        for (int d = 0; d < 3; ++d) {
            a[d] = (long long)floor(u[3 * i + d]);
            fr[d] = u[3 * i + d] - (double)a[d];
            fl[d] = 1.0 - fr[d];
        }
        for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx) {
                    double wt = (dx ? fr[0] : fl[0]) * (dy ? fr[1] : fl[1]) * (dz ? fr[2] : fl[2]);
                    long long x = imod(a[0] + dx, n_fft), y = imod(a[1] + dy, n_fft),
                              z = imod(a[2] + dz, n_fft);
                    out[(z * n_fft + y) * n_fft + x] += w[i] * wt;
                }
    }
}

/* Dense ligand occupancy grid (Eq. 10) on the n_fft^3 periodic grid. */
int orc_occ_dense(int n_fft, int n_atoms, const double *u, const double *thr, uint8_t *out) {
    memset(out, 0, (size_t)n_fft * n_fft * n_fft);
    int cap = 1 << 18;
    int *pts = (int *)malloc(sizeof(int) * 3 * cap);
    if (!pts) return -1;
    int np = occ_points(n_atoms, u, thr, pts, cap);
    if (np < 0) {
        free(pts);
        return -1;
    }
    if (np > cap) np = cap;
    for (int p = 0; p < np; ++p) {
        long long x = imod(pts[3 * p], n_fft), y = imod(pts[3 * p + 1], n_fft),
                  z = imod(pts[3 * p + 2], n_fft);
        out[(z * n_fft + y) * n_fft + x] = 1;
    }
    free(pts);
    return np;
}
