/*
 * FP64 CPU oracle for single-pass raycasting of structured AMR data.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the HIP
 * library is checked against.  It shares no code with the library: only the tests,
 * the smoke check and the CPU-baseline leg of the benchmark load it.
 *
 * What it computes, and where the paper defines it:
 *   - data model: nested subgrids, h^l = h^(l-1)/r                       (Section 3)
 *   - per-pixel rays, ray/kD-leaf segments processed front to back,
 *     per-segment sampling with a step proportional to the level's cell
 *     size, colour/opacity accumulation, one write per pixel           (Section 4 outline, 5.3)
 *   - cell-centred data; interpolation across patch interfaces needs a
 *     shared layer of samples at brick boundaries                      (Section 5 intro)
 *   - vertex-centred data: trilinear interpolation of vertex samples, the
 *     samples at dangling nodes replaced by the coarse interpolant       (Section 5)
 *   - out-of-core subsets: leaves of absent subgrids drawn from the finest
 *     present subgrid holding them                                       (Sections 5.2, 7)
 *   - gradient lighting with gradients taken on the fly, also across
 *     blocks of different subgrids                                      (Section 5, Section 6)
 *   - emission-absorption model                                          (Section 6)
 * Everything the paper leaves open is fixed by the readings documented in the design
 * notes (rays, leaf segments by brute force, midpoint sampling, ghost cells g1-g4,
 * LUT lerp, extinction per unit length, premultiplied colour, early termination).
 *
 * Segments are found by brute force: every leaf box is intersected with the ray by the
 * slab method, leaves are ordered by exit distance and each entry is set to the
 * previous exit.  The field at any point is the trilinear interpolant of the finest
 * patch containing it (found by scanning patches), with ghost values defined
 * recursively.  Compile with -ffp-contract=off: the FP64 ray, plane and sample-position
 * arithmetic is a fixed sequence of correctly rounded operations.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef struct {
    double eye[3], u[3], v[3], w[3];
    double tan_half_fov;
    double win[2];
    int32_t ortho, width, height, pad;
} orc_camera;

typedef struct {
    double v_lo, v_hi, step_frac;
    double t_min;
    double light[3];
    double k_a, k_d, eps_g;
    double clip_lo[3], clip_hi[3];
    int32_t uniform_step, lighting;
    int32_t interp, pad_;       /* 0 trilinear (ghosts g1-g4), 1 nearest cell */
    double lod;                 /* level of detail (Section 4.1, kind-(a) nodes): a node is
                                   rendered from its coarse patch when that patch's cells
                                   project to fewer than lod pixels; 0 disables */
} orc_params;

typedef struct {
    int32_t leaf, patch, n, level;
    double ta, tb;
} orc_seg;

#define NB 16   /* bins per axis of the patch lookup grid */

typedef struct {
    double origin[3], h0[3], hf[3];
    int r, nlev, lmax;
    int np;
    int64_t *plev, *plo, *pdims, *gplo, *gphi;   /* per patch: level; lo/dims (level units); finest box */
    const float *cells;
    int64_t *poff;
    double *hl;          /* [nlev][3] spacing of level l */
    double *hs;          /* [nlev]    step spacing min_a h^l_a */
    int64_t *rpow;       /* [nlev]    r^l */
    int64_t Blo[3], Bhi[3];
    double Bw_lo[3], Bw_hi[3];
    int nl;
    int64_t *leaf;       /* [nl][8] lo3 hi3 patch level */
    double *lw;          /* [nl][6] world planes */
    double **ghost;      /* lazily built padded FP64 bricks (interior + ghost shell) */
    omp_lock_t *locks;
    int **cand;          /* per patch: patches whose boxes meet the 1-cell dilated box */
    int *ncand;
    int *bin_start, *bin_list;   /* patch lookup bins (conservative) */
    int na;              /* kind-(a) nodes, in the tree's pre-order */
    int64_t *anode;      /* [na][9] lo3 hi3 (finest units), cover patch, cover level, depth */
    double *aw;          /* [na][6] world planes */
    uint8_t *res;        /* resident subset (NULL: every patch), out-of-core rendering */
    int *lremap;         /* with res: per leaf, the finest resident patch holding the leaf box */
    int *aremap;         /* with res: the same for the kind-(a) nodes */
    int vertex;          /* 1: vertex-centred data, (n+1)^3 samples per patch */
    double **vfix;       /* vertex mode: per patch, the samples after the dangling-node fix */
} Orc;

static int64_t ipow(int64_t b, int e) { int64_t r = 1; while (e-- > 0) r *= b; return r; }

/* World coordinate of a plane at integer finest-grid coordinate G on axis a. */
static double plane(const Orc *O, int a, int64_t G) {
    double g = (double)G;
    double m = g * O->hf[a];
    return O->origin[a] + m;
}

static int64_t floordiv(int64_t a, int64_t b) { int64_t q = a / b; if ((a % b != 0) && ((a < 0) != (b < 0))) q--; return q; }

void orc_destroy(Orc *O);

Orc *orc_create(const double *origin, const double *h0, int r, int nlev,
                int np, const int64_t *pmeta /* [np][7] level lo3 dims3 */,
                const int64_t *poff, const float *cells,
                int nl, const int64_t *leaves /* [nl][8] */) {
    Orc *O = (Orc *)calloc(1, sizeof(Orc));
    O->r = r; O->nlev = nlev; O->lmax = nlev - 1; O->np = np; O->nl = nl; O->cells = cells;
    O->rpow = (int64_t *)malloc(sizeof(int64_t) * nlev);
    O->hl = (double *)malloc(sizeof(double) * 3 * nlev);
    O->hs = (double *)malloc(sizeof(double) * nlev);
    for (int l = 0; l < nlev; l++) O->rpow[l] = ipow(r, l);
    double hmin = h0[0];
    if (h0[1] < hmin) hmin = h0[1];
    if (h0[2] < hmin) hmin = h0[2];
    for (int a = 0; a < 3; a++) {
        O->origin[a] = origin[a]; O->h0[a] = h0[a];
        O->hf[a] = h0[a] / (double)O->rpow[O->lmax];
        for (int l = 0; l < nlev; l++) O->hl[3 * l + a] = h0[a] / (double)O->rpow[l];
    }
    for (int l = 0; l < nlev; l++) O->hs[l] = hmin / (double)O->rpow[l];
    O->plev = (int64_t *)malloc(sizeof(int64_t) * np);
    O->plo = (int64_t *)malloc(sizeof(int64_t) * 3 * np);
    O->pdims = (int64_t *)malloc(sizeof(int64_t) * 3 * np);
    O->gplo = (int64_t *)malloc(sizeof(int64_t) * 3 * np);
    O->gphi = (int64_t *)malloc(sizeof(int64_t) * 3 * np);
    O->poff = (int64_t *)malloc(sizeof(int64_t) * np);
    int first0 = 1;
    for (int p = 0; p < np; p++) {
        O->plev[p] = pmeta[7 * p];
        int64_t s = O->rpow[O->lmax - O->plev[p]];
        for (int a = 0; a < 3; a++) {
            O->plo[3 * p + a] = pmeta[7 * p + 1 + a];
            O->pdims[3 * p + a] = pmeta[7 * p + 4 + a];
            O->gplo[3 * p + a] = O->plo[3 * p + a] * s;
            O->gphi[3 * p + a] = (O->plo[3 * p + a] + O->pdims[3 * p + a]) * s;
        }
        O->poff[p] = poff[p];
        if (O->plev[p] == 0) {
            for (int a = 0; a < 3; a++) {
                if (first0 || O->gplo[3 * p + a] < O->Blo[a]) O->Blo[a] = O->gplo[3 * p + a];
                if (first0 || O->gphi[3 * p + a] > O->Bhi[a]) O->Bhi[a] = O->gphi[3 * p + a];
            }
            first0 = 0;
        }
    }
    for (int a = 0; a < 3; a++) { O->Bw_lo[a] = plane(O, a, O->Blo[a]); O->Bw_hi[a] = plane(O, a, O->Bhi[a]); }
    O->leaf = (int64_t *)malloc(sizeof(int64_t) * 8 * (nl > 0 ? nl : 1));
    O->lw = (double *)malloc(sizeof(double) * 6 * (nl > 0 ? nl : 1));
    memcpy(O->leaf, leaves, sizeof(int64_t) * 8 * nl);
    for (int i = 0; i < nl; i++)
        for (int a = 0; a < 3; a++) {
            O->lw[6 * i + a] = plane(O, a, O->leaf[8 * i + a]);
            O->lw[6 * i + 3 + a] = plane(O, a, O->leaf[8 * i + 3 + a]);
        }
    O->ghost = (double **)calloc(np, sizeof(double *));
    O->locks = (omp_lock_t *)malloc(sizeof(omp_lock_t) * np);
    for (int p = 0; p < np; p++) omp_init_lock(&O->locks[p]);
    /* candidate lists: patches whose box meets p's box dilated by one level-l cell */
    O->cand = (int **)calloc(np, sizeof(int *));
    O->ncand = (int *)calloc(np, sizeof(int));
    for (int p = 0; p < np; p++) {
        int64_t s = O->rpow[O->lmax - O->plev[p]];
        int cap = 16, n = 0;
        int *lst = (int *)malloc(sizeof(int) * cap);
        for (int q = 0; q < np; q++) {
            int meet = 1;
            for (int a = 0; a < 3; a++) {
                int64_t lo = O->gplo[3 * p + a] - s, hi = O->gphi[3 * p + a] + s;
                if (O->gphi[3 * q + a] < lo || O->gplo[3 * q + a] > hi) { meet = 0; break; }
            }
            if (!meet) continue;
            if (n == cap) { cap *= 2; lst = (int *)realloc(lst, sizeof(int) * cap); }
            lst[n++] = q;
        }
        O->cand[p] = lst; O->ncand[p] = n;
    }
    /* lookup bins over B (conservative: each patch is listed in every bin its box touches,
       widened by one bin on each side) */
    int nb3 = NB * NB * NB;
    int *cnt = (int *)calloc(nb3 + 1, sizeof(int));
    int64_t ext[3];
    for (int a = 0; a < 3; a++) ext[a] = O->Bhi[a] - O->Blo[a];
    for (int pass = 0; pass < 2; pass++) {
        if (pass == 1) {
            O->bin_start = (int *)malloc(sizeof(int) * (nb3 + 1));
            O->bin_start[0] = 0;
            for (int b = 0; b < nb3; b++) O->bin_start[b + 1] = O->bin_start[b] + cnt[b];
            O->bin_list = (int *)malloc(sizeof(int) * (O->bin_start[nb3] > 0 ? O->bin_start[nb3] : 1));
            memset(cnt, 0, sizeof(int) * nb3);
        }
        for (int p = 0; p < np; p++) {
            int b0[3], b1[3];
            for (int a = 0; a < 3; a++) {
                int64_t lo = floordiv((O->gplo[3 * p + a] - O->Blo[a]) * NB, ext[a]) - 1;
                int64_t hi = floordiv((O->gphi[3 * p + a] - O->Blo[a]) * NB, ext[a]) + 1;
                b0[a] = (int)(lo < 0 ? 0 : (lo > NB - 1 ? NB - 1 : lo));
                b1[a] = (int)(hi < 0 ? 0 : (hi > NB - 1 ? NB - 1 : hi));
            }
            for (int z = b0[2]; z <= b1[2]; z++)
                for (int y = b0[1]; y <= b1[1]; y++)
                    for (int x = b0[0]; x <= b1[0]; x++) {
                        int b = x + NB * (y + NB * z);
                        if (pass == 1) O->bin_list[O->bin_start[b] + cnt[b]] = p;
                        cnt[b]++;
                    }
        }
    }
    free(cnt);
    return O;
}

void orc_destroy(Orc *O) {
    if (!O) return;
    for (int p = 0; p < O->np; p++) { free(O->ghost[p]); free(O->cand[p]); omp_destroy_lock(&O->locks[p]); }
    free(O->ghost); free(O->cand); free(O->ncand); free(O->locks);
    free(O->plev); free(O->plo); free(O->pdims); free(O->gplo); free(O->gphi); free(O->poff);
    free(O->hl); free(O->hs); free(O->rpow); free(O->leaf); free(O->lw);
    free(O->bin_start); free(O->bin_list);
    free(O->anode); free(O->aw);
    if (O->vfix) { for (int p = 0; p < O->np; p++) free(O->vfix[p]); free(O->vfix); }
    free(O->res); free(O->lremap); free(O->aremap);
    free(O);
}

/* The kind-(a) nodes (internal nodes inside one subgrid whose cells are all refined further,
 * Section 4.1) that a level-of-detail render may stop at. */
void orc_set_lod_nodes(Orc *O, int na, const int64_t *recs) {
    free(O->anode); free(O->aw);
    O->na = na;
    O->anode = (int64_t *)malloc(sizeof(int64_t) * 9 * (na > 0 ? na : 1));
    O->aw = (double *)malloc(sizeof(double) * 6 * (na > 0 ? na : 1));
    memcpy(O->anode, recs, sizeof(int64_t) * 9 * na);
    for (int i = 0; i < na; i++)
        for (int a = 0; a < 3; a++) {
            O->aw[6 * i + a] = plane(O, a, O->anode[9 * i + a]);
            O->aw[6 * i + 3 + a] = plane(O, a, O->anode[9 * i + 3 + a]);
        }
}

/* Out-of-core rendering (the motive for per-subgrid storage, Sections 5.2 and 7): only the
 * patches with res[p] != 0 are on the device.  Every leaf (and kind-(a) node) keeps its place
 * in the tree but takes its data from the finest resident patch whose box holds the leaf's
 * whole box, at that patch's level and step; a leaf with no resident holder is empty.  The
 * field at a point (gradient taps) is the finest resident patch holding the point.  Ghost
 * values and vertex samples stay those of the full hierarchy (they belong to the bricks).
 * Must follow orc_set_lod_nodes. */
static int box_holds(const Orc *O, int q, const int64_t *lo, const int64_t *hi) {
    for (int a = 0; a < 3; a++)
        if (lo[a] < O->gplo[3 * q + a] || hi[a] > O->gphi[3 * q + a]) return 0;
    return 1;
}

static int resident_holder(const Orc *O, const int64_t *lo, const int64_t *hi) {
    int best = -1;
    for (int q = 0; q < O->np; q++)
        if (O->res[q] && box_holds(O, q, lo, hi) && (best < 0 || O->plev[q] > O->plev[best])) best = q;
    return best;
}

void orc_set_resident(Orc *O, const uint8_t *mask) {
    free(O->res); free(O->lremap); free(O->aremap);
    O->res = (uint8_t *)malloc(O->np > 0 ? O->np : 1);
    memcpy(O->res, mask, O->np);
    O->lremap = (int *)malloc(sizeof(int) * (O->nl > 0 ? O->nl : 1));
    O->aremap = (int *)malloc(sizeof(int) * (O->na > 0 ? O->na : 1));
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < O->nl; i++) {
        const int64_t *L = &O->leaf[8 * i];
        int p = (int)L[6];
        O->lremap[i] = p < 0 ? -1 : (O->res[p] ? p : resident_holder(O, L, L + 3));
    }
    for (int i = 0; i < O->na; i++) {
        const int64_t *A = &O->anode[9 * i];
        int p = (int)A[6];
        O->aremap[i] = O->res[p] ? p : resident_holder(O, A, A + 3);
    }
}

/* ------------------------------------------------------------------------------------ */
/* Field values: interior cells, ghost cells (g1-g4), trilinear interpolation            */
/* ------------------------------------------------------------------------------------ */

static double cell(const Orc *O, int p, int64_t i, int64_t j, int64_t k) {
    const int64_t *n = &O->pdims[3 * p];
    return (double)O->cells[O->poff[p] + i + n[0] * (j + n[1] * k)];
}

static void ensure_ghosts(Orc *O, int p);

/* Value of patch p at index (i,j,k) with -1 <= index <= n on each axis. */
static double pval(Orc *O, int p, int64_t i, int64_t j, int64_t k) {
    const int64_t *n = &O->pdims[3 * p];
    if (i >= 0 && j >= 0 && k >= 0 && i < n[0] && j < n[1] && k < n[2]) return cell(O, p, i, j, k);
    ensure_ghosts(O, p);
    int64_t px = n[0] + 2, py = n[1] + 2;
    return O->ghost[p][(i + 1) + px * ((j + 1) + py * (k + 1))];
}

static double lerp(double a, double b, double f) { return a + f * (b - a); }

/* Trilinear value of patch p at base index i0 with fractions f (lerp x, then y, then z). */
static double trilin(Orc *O, int p, const int64_t i0[3], const double f[3]) {
    double v[8];
    for (int c = 0; c < 8; c++)
        v[c] = pval(O, p, i0[0] + (c & 1), i0[1] + ((c >> 1) & 1), i0[2] + ((c >> 2) & 1));
    double c00 = lerp(v[0], v[1], f[0]), c10 = lerp(v[2], v[3], f[0]);
    double c01 = lerp(v[4], v[5], f[0]), c11 = lerp(v[6], v[7], f[0]);
    double c0 = lerp(c00, c10, f[1]), c1 = lerp(c01, c11, f[1]);
    return lerp(c0, c1, f[2]);
}

/* Is the point with doubled finest coordinates c2 inside patch q (half open)? */
static int contains2(const Orc *O, int q, const int64_t c2[3]) {
    for (int a = 0; a < 3; a++)
        if (c2[a] < 2 * O->gplo[3 * q + a] || c2[a] >= 2 * O->gphi[3 * q + a]) return 0;
    return 1;
}

/* Ghost value of patch p (level l) at ghost index idx (definitions g1-g4). */
static double ghost_value(Orc *O, int p, const int64_t idx[3]) {
    int l = (int)O->plev[p];
    int64_t S = O->rpow[O->lmax - l];
    int64_t c2[3];
    for (int a = 0; a < 3; a++) c2[a] = (2 * (O->plo[3 * p + a] + idx[a]) + 1) * S;
    for (int attempt = 0; attempt < 2; attempt++) {
        /* g1: another patch of the same level holds this cell */
        for (int ci = 0; ci < O->ncand[p]; ci++) {
            int q = O->cand[p][ci];
            if (O->plev[q] != l || !contains2(O, q, c2)) continue;
            int64_t m[3];
            for (int a = 0; a < 3; a++) m[a] = (c2[a] / S - 1) / 2 - O->plo[3 * q + a];
            return cell(O, q, m[0], m[1], m[2]);
        }
        /* g2: outside B -> clamp the centre into B and try again */
        int outside = 0;
        for (int a = 0; a < 3; a++) {
            int64_t lo = 2 * O->Blo[a] + S, hi = 2 * O->Bhi[a] - S;
            if (c2[a] < lo) { c2[a] = lo; outside = 1; }
            if (c2[a] > hi) { c2[a] = hi; outside = 1; }
        }
        if (outside && attempt == 0) continue;
        /* g3: trilinear value of the finest coarser patch containing the centre */
        int best = -1;
        for (int ci = 0; ci < O->ncand[p]; ci++) {
            int q = O->cand[p][ci];
            if (O->plev[q] >= l || !contains2(O, q, c2)) continue;
            if (best < 0 || O->plev[q] > O->plev[best]) best = q;
        }
        if (best >= 0) {
            int64_t Sm = O->rpow[O->lmax - O->plev[best]];
            int64_t i0[3]; double f[3];
            for (int a = 0; a < 3; a++) {
                int64_t num = c2[a] - 2 * O->gplo[3 * best + a] - Sm, den = 2 * Sm;
                i0[a] = floordiv(num, den);
                f[a] = (double)(num - i0[a] * den) / (double)den;
            }
            return trilin(O, best, i0, f);
        }
        break;
    }
    /* g4: no coarser data -> nearest interior cell of p */
    int64_t m[3];
    for (int a = 0; a < 3; a++) {
        m[a] = idx[a];
        if (m[a] < 0) m[a] = 0;
        if (m[a] > O->pdims[3 * p + a] - 1) m[a] = O->pdims[3 * p + a] - 1;
    }
    return cell(O, p, m[0], m[1], m[2]);
}

static void ensure_ghosts(Orc *O, int p) {
    double *g;
#pragma omp atomic read
    g = O->ghost[p];
    if (g) return;
    omp_set_lock(&O->locks[p]);
    if (!O->ghost[p]) {
        const int64_t *n = &O->pdims[3 * p];
        int64_t px = n[0] + 2, py = n[1] + 2, pz = n[2] + 2;
        double *buf = (double *)malloc(sizeof(double) * px * py * pz);
        for (int64_t k = -1; k <= n[2]; k++)
            for (int64_t j = -1; j <= n[1]; j++)
                for (int64_t i = -1; i <= n[0]; i++) {
                    double v;
                    if (i >= 0 && j >= 0 && k >= 0 && i < n[0] && j < n[1] && k < n[2]) v = cell(O, p, i, j, k);
                    else { int64_t idx[3] = {i, j, k}; v = ghost_value(O, p, idx); }
                    buf[(i + 1) + px * ((j + 1) + py * (k + 1))] = v;
                }
#pragma omp atomic write
        O->ghost[p] = buf;
    }
    omp_unset_lock(&O->locks[p]);
}

/* ------------------------------------------------------------------------------------ */
/* Vertex-centred data (Section 5): the samples sit on the grid vertices, a patch of n     */
/* cells holds n+1 per axis, the field is their trilinear interpolant, and samples on a    */
/* patch face that abuts coarser data (dangling nodes) are replaced by the interpolated    */
/* value of the abutting coarse patch, so the field is continuous across the interface.   */
/* ------------------------------------------------------------------------------------ */

static double vsample(const Orc *O, int p, int64_t i, int64_t j, int64_t k) {
    const int64_t *n = &O->pdims[3 * p];
    return O->vfix[p][i + (n[0] + 1) * (j + (n[1] + 1) * k)];
}

/* Trilinear value of patch p's (fixed) vertex samples at vertex index position i0 + f. */
static double vtrilin(const Orc *O, int p, const int64_t i0[3], const double f[3]) {
    double v[8];
    for (int c = 0; c < 8; c++)
        v[c] = vsample(O, p, i0[0] + (c & 1), i0[1] + ((c >> 1) & 1), i0[2] + ((c >> 2) & 1));
    double c00 = lerp(v[0], v[1], f[0]), c10 = lerp(v[2], v[3], f[0]);
    double c01 = lerp(v[4], v[5], f[0]), c11 = lerp(v[6], v[7], f[0]);
    double c0 = lerp(c00, c10, f[1]), c1 = lerp(c01, c11, f[1]);
    return lerp(c0, c1, f[2]);
}

/* Value of patch p's vertex data at the point with finest-level coordinates G (a point of
   p's closed box): level-p vertex position (G - lo) / S, the base index kept in [0, n-1]. */
static double vertex_at_G(const Orc *O, int p, const int64_t G[3]) {
    int64_t S = O->rpow[O->lmax - O->plev[p]];
    int64_t i0[3]; double f[3];
    for (int a = 0; a < 3; a++) {
        int64_t num = G[a] - O->gplo[3 * p + a];
        int64_t i = floordiv(num, S), n = O->pdims[3 * p + a];
        if (i > n - 1) i = n - 1;
        if (i < 0) i = 0;
        i0[a] = i;
        f[a] = (double)(num - i * S) / (double)S;
    }
    return vtrilin(O, p, i0, f);
}

int orc_locate(Orc *O, const double *x, int brute);

/* Switches the oracle to vertex-centred data and applies the dangling-node fix.  For every
 * vertex on the boundary of a level-l patch, the eight finest-level cells around it that lie
 * in B are each owned by the finest patch holding them (the patch located at the cell's
 * centre); if the coarsest such owner is coarser than l, the sample becomes that owner's
 * interpolated value at the vertex (the first owner of that level in the octant order, bit a
 * of the octant number set for the + side of axis a).  Levels are fixed coarsest first, so
 * coarse values are final before finer patches read them. */
void orc_set_vertex(Orc *O) {
    O->vertex = 1;
    O->vfix = (double **)calloc(O->np, sizeof(double *));
    for (int l = 0; l <= O->lmax; l++) {
#pragma omp parallel for schedule(dynamic)
        for (int p = 0; p < O->np; p++) {
            if (O->plev[p] != l) continue;
            const int64_t *n = &O->pdims[3 * p];
            const int64_t nx = n[0] + 1, ny = n[1] + 1, nz = n[2] + 1;
            const int64_t S = O->rpow[O->lmax - l];
            double *buf = (double *)malloc(sizeof(double) * nx * ny * nz);
            for (int64_t k = 0; k < nz; k++)
                for (int64_t j = 0; j < ny; j++)
                    for (int64_t i = 0; i < nx; i++) {
                        const int64_t idx = i + nx * (j + ny * k);
                        buf[idx] = (double)O->cells[O->poff[p] + idx];
                        const int on_face = i == 0 || j == 0 || k == 0 || i == n[0] || j == n[1] || k == n[2];
                        if (!on_face) continue;
                        const int64_t G[3] = {O->gplo[3 * p] + i * S, O->gplo[3 * p + 1] + j * S,
                                              O->gplo[3 * p + 2] + k * S};
                        int m = l, own = -1;
                        for (int s = 0; s < 8; s++) {
                            double xc[3];   /* centre of the finest cell on side s of the vertex */
                            int inB = 1;
                            for (int a = 0; a < 3; a++) {
                                int64_t c = ((s >> a) & 1) ? G[a] : G[a] - 1;
                                if (c < O->Blo[a] || c >= O->Bhi[a]) inB = 0;
                                xc[a] = plane(O, a, c) + 0.5 * O->hf[a];
                            }
                            if (!inB) continue;
                            int q = orc_locate(O, xc, 0);
                            if (q >= 0 && O->plev[q] < m) { m = (int)O->plev[q]; own = q; }
                        }
                        if (own >= 0) buf[idx] = vertex_at_G(O, own, G);
                    }
            O->vfix[p] = buf;
        }
    }
}

/* Sample of patch p after the fix, at vertex index (i, j, k) (0 <= index <= n). */
double orc_vertex_value(Orc *O, int p, int64_t i, int64_t j, int64_t k) { return vsample(O, p, i, j, k); }

/* Trilinear value of patch p's vertex data at world point x: q = (x - lo) / h, the base index
   kept in [0, n-1] (a point on the upper face uses the last cell with weight 1). */
static double vertex_in(Orc *O, int p, const double x[3]) {
    int l = (int)O->plev[p];
    int64_t i0[3]; double f[3];
    for (int a = 0; a < 3; a++) {
        double lo = plane(O, a, O->gplo[3 * p + a]);
        double q = (x[a] - lo) / O->hl[3 * l + a];
        double fl = floor(q);
        int64_t n = O->pdims[3 * p + a];
        int64_t i = (int64_t)fl;
        if (i > n - 1) i = n - 1;
        if (i < 0) i = 0;
        i0[a] = i;
        f[a] = q - (double)i;
    }
    return vtrilin(O, p, i0, f);
}

/* Does patch q contain world point x?  Half-open boxes, except that B's upper faces
   count as inside. */
static int contains_world(const Orc *O, int q, const double x[3]) {
    for (int a = 0; a < 3; a++) {
        double lo = plane(O, a, O->gplo[3 * q + a]), hi = plane(O, a, O->gphi[3 * q + a]);
        if (x[a] < lo) return 0;
        if (x[a] >= hi && !(x[a] == hi && O->gphi[3 * q + a] == O->Bhi[a])) return 0;
    }
    return 1;
}

static int in_B(const Orc *O, const double x[3]) {
    for (int a = 0; a < 3; a++) if (x[a] < O->Bw_lo[a] || x[a] > O->Bw_hi[a]) return 0;
    return 1;
}

/* Finest patch containing x (ties impossible: same-level patches are disjoint); -1 if none. */
int orc_locate(Orc *O, const double *x, int brute) {
    if (!in_B(O, x)) return -1;
    int best = -1;
    if (brute) {
        for (int q = 0; q < O->np; q++)
            if ((!O->res || O->res[q]) && contains_world(O, q, x) && (best < 0 || O->plev[q] > O->plev[best])) best = q;
        return best;
    }
    int b[3];
    for (int a = 0; a < 3; a++) {
        double t = (x[a] - O->Bw_lo[a]) / (O->Bw_hi[a] - O->Bw_lo[a]) * NB;
        int bi = (int)floor(t);
        b[a] = bi < 0 ? 0 : (bi > NB - 1 ? NB - 1 : bi);
    }
    int bin = b[0] + NB * (b[1] + NB * b[2]);
    for (int s = O->bin_start[bin]; s < O->bin_start[bin + 1]; s++) {
        int q = O->bin_list[s];
        if (O->res && !O->res[q]) continue;
        if (contains_world(O, q, x) && (best < 0 || O->plev[q] > O->plev[best])) best = q;
    }
    return best;
}

/* Trilinear value of patch p at world point x. */
static double field_in(Orc *O, int p, const double x[3]) {
    int l = (int)O->plev[p];
    int64_t i0[3]; double f[3];
    for (int a = 0; a < 3; a++) {
        double lo = plane(O, a, O->gplo[3 * p + a]);
        double q = (x[a] - lo) / O->hl[3 * l + a] - 0.5;
        double fl = floor(q);
        i0[a] = (int64_t)fl;
        f[a] = q - fl;
    }
    return trilin(O, p, i0, f);
}

/* Nearest-neighbour value of patch p at world point x (Section 5 samples cell-centred data
 * without interpolation): the value of the interior cell holding x, floor((x - lo) / h), the
 * index clamped into the patch (a point on B's closed upper face lies in the last cell). */
static double nearest_in(Orc *O, int p, const double x[3]) {
    int l = (int)O->plev[p];
    int64_t i[3];
    for (int a = 0; a < 3; a++) {
        double lo = plane(O, a, O->gplo[3 * p + a]);
        int64_t c = (int64_t)floor((x[a] - lo) / O->hl[3 * l + a]);
        int64_t n = O->pdims[3 * p + a];
        i[a] = c < 0 ? 0 : (c >= n ? n - 1 : c);
    }
    return cell(O, p, i[0], i[1], i[2]);
}

static double value_in(Orc *O, int p, const double x[3], int interp) {
    if (O->vertex) return vertex_in(O, p, x);
    return interp ? nearest_in(O, p, x) : field_in(O, p, x);
}

/* F(x) with the given interpolation; returns 0 and sets *ok = 0 where no patch holds x. */
double orc_field_mode(Orc *O, const double *x, int interp, int *ok) {
    int p = orc_locate(O, x, 0);
    if (p < 0) { if (ok) *ok = 0; return 0.0; }
    if (ok) *ok = 1;
    return value_in(O, p, x, interp);
}

/* F(x) (trilinear); returns 0 and sets *ok = 0 where no patch holds x. */
double orc_field(Orc *O, const double *x, int *ok) { return orc_field_mode(O, x, 0, ok); }

double orc_patch_value(Orc *O, int p, int64_t i, int64_t j, int64_t k) { return pval(O, p, i, j, k); }

/* ------------------------------------------------------------------------------------ */
/* Rays and segments                                                                     */
/* ------------------------------------------------------------------------------------ */

void orc_ray(const orc_camera *c, int i, int j, double *o, double *d) {
    double s = (double)(2 * i + 1) / (double)c->width - 1.0;
    double t = 1.0 - (double)(2 * j + 1) / (double)c->height;
    double dd[3];
    if (c->ortho) {
        double a = s * c->win[0], b = t * c->win[1];
        for (int k = 0; k < 3; k++) {
            double e = c->eye[k] + a * c->u[k];
            o[k] = e + b * c->v[k];
            dd[k] = c->w[k];
        }
    } else {
        double aspect = (double)c->width / (double)c->height;
        double a = (s * c->tan_half_fov) * aspect, b = t * c->tan_half_fov;
        for (int k = 0; k < 3; k++) {
            o[k] = c->eye[k];
            double e = c->w[k] + a * c->u[k];
            dd[k] = e + b * c->v[k];
        }
    }
    double n2 = dd[0] * dd[0] + dd[1] * dd[1];
    n2 = n2 + dd[2] * dd[2];
    double nr = sqrt(n2);
    for (int k = 0; k < 3; k++) d[k] = dd[k] / nr;
}

/* Clip the ray to B ∩ clip box. Returns 1 on a hit with t0 < t1. */
static int clip_ray(const Orc *O, const orc_params *P, const double o[3], const double d[3], double *t0, double *t1) {
    double lo_t = 0.0, hi_t = INFINITY;
    for (int a = 0; a < 3; a++) {
        double lo = O->Bw_lo[a] > P->clip_lo[a] ? O->Bw_lo[a] : P->clip_lo[a];
        double hi = O->Bw_hi[a] < P->clip_hi[a] ? O->Bw_hi[a] : P->clip_hi[a];
        if (d[a] == 0.0) {
            if (!(o[a] >= lo && o[a] < hi)) return 0;
            continue;
        }
        double inv = 1.0 / d[a];
        double ta = (lo - o[a]) * inv, tb = (hi - o[a]) * inv;
        double tn = ta < tb ? ta : tb, tf = ta < tb ? tb : ta;
        if (tn > lo_t) lo_t = tn;
        if (tf < hi_t) hi_t = tf;
    }
    *t0 = lo_t; *t1 = hi_t;
    return hi_t > lo_t;
}

typedef struct { double te, tx; int leaf; } cand_t;

static int cmp_cand(const void *a, const void *b) {
    const cand_t *x = (const cand_t *)a, *y = (const cand_t *)b;
    if (x->tx < y->tx) return -1;
    if (x->tx > y->tx) return 1;
    return x->leaf - y->leaf;
}

/* All leaf segments along the ray, front to back; returns count (segments written up to cap).
   *flag is set when consecutive leaves do not share an exact entry/exit (ray along an edge). */
static int segments(const Orc *O, const double o[3], const double d[3], double t0, double t1,
                    cand_t *buf, int cap, int *flag) {
    int n = 0;
    double inv[3];
    for (int a = 0; a < 3; a++) inv[a] = d[a] != 0.0 ? 1.0 / d[a] : 0.0;
    for (int i = 0; i < O->nl; i++) {
        double te = t0, tx = t1;
        int miss = 0;
        for (int a = 0; a < 3 && !miss; a++) {
            double lo = O->lw[6 * i + a], hi = O->lw[6 * i + 3 + a];
            if (d[a] == 0.0) { if (!(o[a] >= lo && o[a] < hi)) miss = 1; continue; }
            double ta = (lo - o[a]) * inv[a], tb = (hi - o[a]) * inv[a];
            double tn = ta < tb ? ta : tb, tf = ta < tb ? tb : ta;
            if (tn > te) te = tn;
            if (tf < tx) tx = tf;
        }
        if (miss || !(tx > te)) continue;
        if (n < cap) { buf[n].te = te; buf[n].tx = tx; buf[n].leaf = i; }
        n++;
    }
    if (n > cap) { *flag |= 2; n = cap; }
    qsort(buf, n, sizeof(cand_t), cmp_cand);
    double prev = t0;
    for (int k = 0; k < n; k++) {
        if (buf[k].te != prev) *flag |= 1;
        prev = buf[k].tx;
    }
    if (n > 0 && prev != t1) *flag |= 1;
    return n;
}

/* ------------------------------------------------------------------------------------ */
/* Shading, classification, compositing                                                  */
/* ------------------------------------------------------------------------------------ */

typedef struct {
    int i0; double f;          /* LUT cell and weight */
    double rgb[3], sigma, delta, alpha, T, shade;
    double g[3], dot, den;     /* normalised gradient, g . l, sqrt(|g|^2 + eps^2) */
} sample_t;

static void classify(const double *lut, double F, const orc_params *P, sample_t *s) {
    double u = (F - P->v_lo) / (P->v_hi - P->v_lo);
    if (u < 0.0) u = 0.0;
    if (u > 1.0) u = 1.0;
    double x = 255.0 * u;
    int i0 = (int)floor(x);
    if (i0 > 254) i0 = 254;
    double f = x - (double)i0;
    s->i0 = i0; s->f = f;
    for (int c = 0; c < 3; c++) s->rgb[c] = lerp(lut[4 * i0 + c], lut[4 * (i0 + 1) + c], f);
    s->sigma = lerp(lut[4 * i0 + 3], lut[4 * (i0 + 1) + 3], f);
}

/* The field a gradient tap reads: inside the box of a level-of-detail segment (half-open) the
 * segment's coarse patch, elsewhere the finest data. */
static double tap_field(Orc *O, const orc_params *P, const double *lodbox, int lodp, const double x[3], int *ok) {
    if (lodbox) {
        int in = 1;
        for (int a = 0; a < 3; a++) in = in && x[a] >= lodbox[a] && x[a] < lodbox[3 + a];
        if (in) { *ok = 1; return value_in(O, lodp, x, P->interp); }
    }
    return orc_field_mode(O, x, P->interp, ok);
}

static void shade_sample(Orc *O, const orc_params *P, const double lhat[3], int lev, double F0,
                         const double x[3], const double *lodbox, int lodp, sample_t *s) {
    double range = P->v_hi - P->v_lo;
    for (int a = 0; a < 3; a++) {
        double xp[3] = {x[0], x[1], x[2]}, xm[3] = {x[0], x[1], x[2]};
        xp[a] = x[a] + O->hl[3 * lev + a];
        xm[a] = x[a] - O->hl[3 * lev + a];
        int okp, okm;
        double Fp = tap_field(O, P, lodbox, lodp, xp, &okp), Fm = tap_field(O, P, lodbox, lodp, xm, &okm);
        double g;
        if (okp && okm) g = (Fp - Fm) / (2.0 * range);
        else if (okp) g = (Fp - F0) / range;
        else if (okm) g = (F0 - Fm) / range;
        else g = 0.0;
        s->g[a] = g;
    }
    double dot = s->g[0] * lhat[0] + s->g[1] * lhat[1] + s->g[2] * lhat[2];
    double den = sqrt(s->g[0] * s->g[0] + s->g[1] * s->g[1] + s->g[2] * s->g[2] + P->eps_g * P->eps_g);
    s->dot = dot; s->den = den;
    s->shade = P->k_a + (den > 0.0 ? P->k_d * fabs(dot) / den : 0.0);
}

/* Transmittance from x to a point light at pl (lighting = 2, the secondary rays of the paper's
 * global-illumination example, Section 6): the segment from x to the light, clipped to B, is
 * cut into leaf segments and sampled with the primary rule (midpoints, step proportional to the
 * leaf level's cell size); T_L = exp(-sum sigma_j delta_j). */
static double light_transmittance(Orc *O, const orc_params *P, const double *lut, const double x[3],
                                  const double pl[3]) {
    double v[3], dist2 = 0.0;
    for (int a = 0; a < 3; a++) { v[a] = pl[a] - x[a]; }
    dist2 = v[0] * v[0] + v[1] * v[1];
    dist2 = dist2 + v[2] * v[2];
    double dist = sqrt(dist2);
    if (!(dist > 0.0)) return 1.0;
    double d[3];
    for (int a = 0; a < 3; a++) d[a] = v[a] / dist;
    /* clip [0, dist] to B */
    double lo_t = 0.0, hi_t = dist;
    for (int a = 0; a < 3; a++) {
        double lo = O->Bw_lo[a], hi = O->Bw_hi[a];
        if (d[a] == 0.0) { if (!(x[a] >= lo && x[a] < hi)) return 1.0; continue; }
        double inv = 1.0 / d[a];
        double ta = (lo - x[a]) * inv, tb = (hi - x[a]) * inv;
        double tn = ta < tb ? ta : tb, tf = ta < tb ? tb : ta;
        if (tn > lo_t) lo_t = tn;
        if (tf < hi_t) hi_t = tf;
    }
    if (!(hi_t > lo_t)) return 1.0;
    int cap = 64, flag = 0;
    cand_t *buf = (cand_t *)malloc(sizeof(cand_t) * cap);
    int n = segments(O, x, d, lo_t, hi_t, buf, cap, &flag);
    while (flag & 2) { cap *= 2; buf = (cand_t *)realloc(buf, sizeof(cand_t) * cap); flag = 0; n = segments(O, x, d, lo_t, hi_t, buf, cap, &flag); }
    double tau = 0.0, ta = lo_t;
    for (int k = 0; k < n; k++) {
        double tb = buf[k].tx;
        const int64_t *L = &O->leaf[8 * buf[k].leaf];
        int p = (int)L[6], lev = (int)L[7];
        if (O->res && p >= 0) { p = O->lremap[buf[k].leaf]; if (p >= 0) lev = (int)O->plev[p]; }
        if (p >= 0) {
            int slev = P->uniform_step ? O->lmax : lev;
            double step = P->step_frac * O->hs[slev];
            double nn = ceil((tb - ta) / step - 0x1p-20);
            int64_t ns = nn < 1.0 ? 1 : (int64_t)nn;
            double delta = (tb - ta) / (double)ns;
            for (int64_t j = 0; j < ns; j++) {
                double t = ta + ((double)j + 0.5) * delta;
                double y[3];
                for (int a = 0; a < 3; a++) y[a] = x[a] + t * d[a];
                sample_t sm;
                classify(lut, value_in(O, p, y, P->interp), P, &sm);
                tau += sm.sigma * delta;
            }
        }
        ta = tb;
    }
    free(buf);
    return exp(-tau);
}

/* Walks one ray. Fills rgba; if samples != NULL, appends every evaluated sample to it. */
typedef struct { sample_t *v; int64_t n, cap; } svec;

static void svec_push(svec *s, const sample_t *x) {
    if (s->n == s->cap) { s->cap = s->cap ? 2 * s->cap : 1024; s->v = (sample_t *)realloc(s->v, sizeof(sample_t) * s->cap); }
    s->v[s->n++] = *x;
}

static int walk_ray(Orc *O, const orc_camera *cam, const orc_params *P, const double *lut, int pi, int pj,
                    double rgba[4], int64_t *nsamp, orc_seg *trace, int trace_cap, int *trace_n,
                    svec *samples, cand_t **cbuf, int *ccap) {
    double o[3], d[3], t0, t1;
    int flag = 0;
    orc_ray(cam, pi, pj, o, d);
    rgba[0] = rgba[1] = rgba[2] = rgba[3] = 0.0;
    *nsamp = 0;
    if (trace_n) *trace_n = 0;
    if (!clip_ray(O, P, o, d, &t0, &t1)) return 0;
    int n = segments(O, o, d, t0, t1, *cbuf, *ccap, &flag);
    while (flag & 2) {   /* grow and retry */
        *ccap *= 2; *cbuf = (cand_t *)realloc(*cbuf, sizeof(cand_t) * (*ccap)); flag = 0;
        n = segments(O, o, d, t0, t1, *cbuf, *ccap, &flag);
    }
    double lhat[3] = {0, 0, 0};
    double ln = sqrt(P->light[0] * P->light[0] + P->light[1] * P->light[1] + P->light[2] * P->light[2]);
    if (ln > 0) for (int a = 0; a < 3; a++) lhat[a] = P->light[a] / ln;
    double C[3] = {0, 0, 0}, T = 1.0;
    double ta = t0;
    int done = 0;
    /* level of detail: the kind-(a) nodes the ray crosses, with their slab intervals */
    const int lod_on = P->lod > 0.0 && O->na > 0;
    double pix = 0.0;
    int nA = 0;
    double *aint = NULL;   /* [nA][2] te, tx */
    int *aid = NULL;
    if (lod_on) {
        pix = cam->ortho ? (2.0 * cam->win[1]) / (double)cam->height : (2.0 * cam->tan_half_fov) / (double)cam->height;
        aint = (double *)malloc(sizeof(double) * 2 * O->na);
        aid = (int *)malloc(sizeof(int) * O->na);
        double inv[3];
        for (int a = 0; a < 3; a++) inv[a] = d[a] != 0.0 ? 1.0 / d[a] : 0.0;
        for (int i = 0; i < O->na; i++) {
            double te = t0, tx = t1;
            int miss = 0;
            for (int a = 0; a < 3 && !miss; a++) {
                double lo = O->aw[6 * i + a], hi = O->aw[6 * i + 3 + a];
                if (d[a] == 0.0) { if (!(o[a] >= lo && o[a] < hi)) miss = 1; continue; }
                double tA = (lo - o[a]) * inv[a], tB = (hi - o[a]) * inv[a];
                double tn = tA < tB ? tA : tB, tf = tA < tB ? tB : tA;
                if (tn > te) te = tn;
                if (tf < tx) tx = tf;
            }
            if (miss || !(tx > te)) continue;
            aint[2 * nA] = te; aint[2 * nA + 1] = tx; aid[nA] = i; nA++;
        }
    }
    for (int k = 0; k < n && !done; k++) {
        cand_t *c = &(*cbuf)[k];
        double tb = c->tx;
        const int64_t *L = &O->leaf[8 * c->leaf];
        int p = (int)L[6], lev = (int)L[7];
        if (O->res && p >= 0) { p = O->lremap[c->leaf]; if (p >= 0) lev = (int)O->plev[p]; }
        int seg_id = c->leaf;
        const double *lodbox = NULL;
        if (lod_on) {
            /* the shallowest kind-(a) node holding the ray just after ta whose coarse cells
               project to fewer than lod pixels at ta: render it whole from its cover patch */
            int best = -1;
            for (int q = 0; q < nA; q++) {
                if (!(aint[2 * q] <= ta && ta < aint[2 * q + 1])) continue;
                const int64_t *A = &O->anode[9 * aid[q]];
                int alev = (int)A[7];
                if (O->res) {        /* out-of-core: the node's resident holder, if any */
                    if (O->aremap[aid[q]] < 0) continue;
                    alev = (int)O->plev[O->aremap[aid[q]]];
                }
                double foot = cam->ortho ? pix : ta * pix;
                if (!(O->hs[alev] < P->lod * foot)) continue;
                if (best < 0 || A[8] < O->anode[9 * aid[best] + 8]) best = q;
            }
            if (best >= 0) {
                const int64_t *A = &O->anode[9 * aid[best]];
                tb = aint[2 * best + 1];
                p = (int)A[6];
                lev = (int)A[7];
                if (O->res) { p = O->aremap[aid[best]]; if (p >= 0) lev = (int)O->plev[p]; }
                seg_id = O->nl + aid[best];
                lodbox = &O->aw[6 * aid[best]];
                while (k + 1 < n && (*cbuf)[k + 1].tx <= tb) k++;   /* leaves inside the node */
            }
        }
        int slev = P->uniform_step ? O->lmax : lev;
        double step = P->step_frac * O->hs[slev];
        double ratio = (tb - ta) / step;
        double nn = ceil(ratio - 0x1p-20);
        int64_t ns = nn < 1.0 ? 1 : (int64_t)nn;
        double delta = (tb - ta) / (double)ns;
        if (trace && *trace_n < trace_cap) {
            orc_seg *s = &trace[*trace_n];
            s->leaf = seg_id; s->patch = p; s->n = p >= 0 ? (int)ns : 0; s->level = lev; s->ta = ta; s->tb = tb;
        }
        if (trace_n) (*trace_n)++;
        if (p >= 0) {
            for (int64_t j = 0; j < ns; j++) {
                double t = ta + ((double)j + 0.5) * delta;
                double x[3];
                for (int a = 0; a < 3; a++) x[a] = o[a] + t * d[a];
                double F0 = value_in(O, p, x, P->interp);
                sample_t s;
                classify(lut, F0, P, &s);
                s.delta = delta;
                s.alpha = 1.0 - exp(-s.sigma * delta);
                s.T = T;
                if (P->lighting == 2) {
                    s.g[0] = s.g[1] = s.g[2] = 0; s.dot = 0; s.den = 0;
                    s.shade = P->k_a + P->k_d * light_transmittance(O, P, lut, x, P->light);
                } else if (P->lighting) {
                    shade_sample(O, P, lhat, lev, F0, x, lodbox, p, &s);
                } else { s.shade = 1.0; s.g[0] = s.g[1] = s.g[2] = 0; s.dot = 0; s.den = 0; }
                for (int ch = 0; ch < 3; ch++) C[ch] += T * s.alpha * s.shade * s.rgb[ch];
                T = T * (1.0 - s.alpha);
                (*nsamp)++;
                if (samples) svec_push(samples, &s);
                if (P->t_min > 0.0 && T < P->t_min) { done = 1; break; }
            }
        }
        ta = tb;
    }
    free(aint); free(aid);
    rgba[0] = C[0]; rgba[1] = C[1]; rgba[2] = C[2]; rgba[3] = 1.0 - T;
    return flag;
}

/* Render npix pixels (pix = [npix][2] column, row). Optional per-pixel segment trace
   (trace_cap records per pixel). Returns the number of rays flagged as edge cases. */
int orc_render(Orc *O, const orc_camera *cam, const orc_params *P, const double *lut,
               int64_t npix, const int32_t *pix, double *rgba, int64_t *nsamp,
               orc_seg *trace, int trace_cap, int32_t *trace_n, int32_t *flags) {
    int nflag = 0;
#pragma omp parallel reduction(+ : nflag)
    {
        int ccap = 256;
        cand_t *cbuf = (cand_t *)malloc(sizeof(cand_t) * ccap);
#pragma omp for schedule(dynamic, 16)
        for (int64_t q = 0; q < npix; q++) {
            int tn = 0;
            int f = walk_ray(O, cam, P, lut, pix[2 * q], pix[2 * q + 1], &rgba[4 * q], &nsamp[q],
                             trace ? &trace[q * trace_cap] : NULL, trace_cap, &tn, NULL, &cbuf, &ccap);
            if (trace_n) trace_n[q] = tn;
            if (flags) flags[q] = f;
            if (f & 1) nflag++;
        }
        free(cbuf);
    }
    return nflag;
}

/* Reverse mode: given dL/dRGBA per pixel, accumulate dL/dLUT [256][4] and
   dL/d(light_x, light_y, light_z, k_a, k_d). */
void orc_grad(Orc *O, const orc_camera *cam, const orc_params *P, const double *lut,
              int64_t npix, const int32_t *pix, const double *grad_rgba,
              double *grad_lut, double *grad_light) {
    int nt = omp_get_max_threads();
    double *acc = (double *)calloc((size_t)nt * 1029, sizeof(double));
    double ln = sqrt(P->light[0] * P->light[0] + P->light[1] * P->light[1] + P->light[2] * P->light[2]);
    double lhat[3] = {0, 0, 0};
    if (ln > 0) for (int a = 0; a < 3; a++) lhat[a] = P->light[a] / ln;
#pragma omp parallel
    {
        double *my = &acc[(size_t)omp_get_thread_num() * 1029];
        svec S = {0, 0, 0};
        int ccap = 256;
        cand_t *cbuf = (cand_t *)malloc(sizeof(cand_t) * ccap);
#pragma omp for schedule(dynamic, 16)
        for (int64_t q = 0; q < npix; q++) {
            double rgba[4]; int64_t ns;
            S.n = 0;
            walk_ray(O, cam, P, lut, pix[2 * q], pix[2 * q + 1], rgba, &ns, NULL, 0, NULL, &S, &cbuf, &ccap);
            const double *gC = &grad_rgba[4 * q];
            double gA = grad_rgba[4 * q + 3];
            double TN = 1.0 - rgba[3];
            if (S.n > 0) {
                const sample_t *last = &S.v[S.n - 1];
                TN = last->T * (1.0 - last->alpha);
            }
            double rest[3] = {0, 0, 0};      /* sum over later samples of T_j alpha_j e_j */
            for (int64_t k = S.n - 1; k >= 0; k--) {
                const sample_t *s = &S.v[k];
                double Tn = s->T * (1.0 - s->alpha);
                double e[3], dsig = 0.0, dshade = 0.0;
                for (int c = 0; c < 3; c++) {
                    e[c] = s->shade * s->rgb[c];
                    dsig += gC[c] * (Tn * e[c] - rest[c]);
                }
                dsig = s->delta * (dsig + gA * TN);
                double w = s->T * s->alpha;
                for (int c = 0; c < 3; c++) {
                    double drgb = gC[c] * w * s->shade;
                    my[4 * s->i0 + c] += (1.0 - s->f) * drgb;
                    my[4 * (s->i0 + 1) + c] += s->f * drgb;
                    dshade += gC[c] * w * s->rgb[c];
                }
                my[4 * s->i0 + 3] += (1.0 - s->f) * dsig;
                my[4 * (s->i0 + 1) + 3] += s->f * dsig;
                if (P->lighting && s->den > 0.0) {
                    double sg = s->dot > 0 ? 1.0 : (s->dot < 0 ? -1.0 : 0.0);
                    for (int a = 0; a < 3; a++) {
                        double dl = P->k_d * sg / s->den * (s->g[a] - s->dot * lhat[a]) / ln;
                        my[1024 + a] += dshade * dl;
                    }
                    my[1027] += dshade;
                    my[1028] += dshade * fabs(s->dot) / s->den;
                } else if (P->lighting) {
                    my[1027] += dshade;
                }
                for (int c = 0; c < 3; c++) rest[c] += w * e[c];
            }
        }
        free(S.v);
        free(cbuf);
    }
    for (int i = 0; i < 1029; i++) {
        double s = 0;
        for (int t = 0; t < nt; t++) s += acc[(size_t)t * 1029 + i];
        if (i < 1024) grad_lut[i] = s; else grad_light[i - 1024] = s;
    }
    free(acc);
}

int orc_num_threads(void) { return omp_get_max_threads(); }
