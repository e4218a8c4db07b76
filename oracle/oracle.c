/*
 * oracle.c -- plain CPU evaluator of SLCS formulas over 2-D images.
 *
 * TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may build, load or
 * call this file.  It shares no code, header, table or helper with the GPU
 * library, and it never calls it.
 *
 * Data: a mask is one byte per pixel (0 or 1), row-major [H][W].  An image is
 * channel-planar [C][H][W], float32 or uint8, with no row padding.
 *
 * What is computed (paper "A spatial model checker in GPU", Sect. 2):
 *   p            threshold atom on a pixel feature (intensity of a channel);
 *   !a, a & b    pixel-wise complement and intersection (Sect. 2, Boolean
 *                operators); a | b is !(!a & !b), computed directly;
 *   N a          Moore-neighbourhood dilation: pixels sharing an edge or a
 *                vertex with a pixel of a, the pixel itself included;
 *   rho a[b]     pixels x with a path pi and an index l >= 0 such that
 *                pi_0 = x, pi_l satisfies a, and pi_1 .. pi_{l-1} satisfy b
 *                (Eq. def:syntax and the reachability paragraph after it);
 *   interior a   erosion, derived as !N!a (Sect. 2, derived operators);
 *   surrounded(a,b)  a & !rho(!a & !b)[!b]: x satisfies a and no path from
 *                x reaches a pixel outside a while avoiding b at every index
 *                after 0 (surroundedness derived from reachability, Sect. 2);
 *   grow(a,b)    a | (b & rho a[b]): a, plus every 8-connected region of b
 *                that touches N a (the operator of Fig. specification and
 *                the prose under it, Sect. 4.2).
 *
 * Pixels outside the image do not exist: N never reaches past the border and
 * paths stay inside the image.  Paths are 8-connected (Moore neighbourhood).
 *
 * reach is evaluated as a breadth-first flood: start from every pixel of a,
 * step only onto 8-neighbours that satisfy b, then dilate the flooded set
 * once.  A pixel x is in rho a[b] iff x is the flooded set's neighbour or
 * member: pi_1 .. pi_{l-1} are exactly the flood's b-steps back from pi_l.
 *
 * Threshold constants are read as double and rounded once to float32; pixels
 * are converted to float32 (exact for uint8) and compared in float32.
 * percentile(img, c, q) is the k-th smallest value of channel c over all H*W
 * pixels, k = clamp(ceil(q * n) - 1, 0, n - 1), nearest rank, no
 * interpolation (the paper names a percentiles operator but does not define
 * it).
 */
#include <ctype.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_EPARSE (-2)
#define ORC_ESHAPE (-3)
#define ORC_ENOMEM (-4)

#define DT_F32 0
#define DT_U8 1
#define DT_U16 2 /* the paper's pixel type (Sect. 3 restricts its tool to 2-D uint16 images) */

/* ------------------------------------------------------------------ */
/* Primitive operators on byte masks                                   */
/* ------------------------------------------------------------------ */

void oracle_not(const uint8_t *a, int64_t n, uint8_t *out)
{
    for (int64_t i = 0; i < n; i++)
        out[i] = a[i] ? 0 : 1;
}

void oracle_and(const uint8_t *a, const uint8_t *b, int64_t n, uint8_t *out)
{
    for (int64_t i = 0; i < n; i++)
        out[i] = (a[i] && b[i]) ? 1 : 0;
}

void oracle_or(const uint8_t *a, const uint8_t *b, int64_t n, uint8_t *out)
{
    for (int64_t i = 0; i < n; i++)
        out[i] = (a[i] || b[i]) ? 1 : 0;
}

/* N a: (y,x) is set iff a pixel of a lies in the 3x3 block centred on (y,x),
 * counting only pixels inside the image. */
void oracle_near(const uint8_t *a, int H, int W, uint8_t *out)
{
    for (int y = 0; y < H; y++) {
        for (int x = 0; x < W; x++) {
            int v = 0;
            for (int dy = -1; dy <= 1 && !v; dy++) {
                for (int dx = -1; dx <= 1; dx++) {
                    int yy = y + dy, xx = x + dx;
                    if (yy < 0 || yy >= H || xx < 0 || xx >= W)
                        continue;
                    if (a[(int64_t)yy * W + xx]) {
                        v = 1;
                        break;
                    }
                }
            }
            out[(int64_t)y * W + x] = (uint8_t)v;
        }
    }
}

/* rho a[b] by breadth-first flood from a through b, then one dilation. */
int oracle_reach(const uint8_t *a, const uint8_t *b, int H, int W, uint8_t *out)
{
    int64_t n = (int64_t)H * W;
    if (n == 0)
        return ORC_OK;
    uint8_t *mark = (uint8_t *)calloc((size_t)n, 1);
    int64_t *queue = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!mark || !queue) {
        free(mark);
        free(queue);
        return ORC_ENOMEM;
    }
    int64_t head = 0, tail = 0;
    for (int64_t p = 0; p < n; p++) {
        if (a[p]) {
            mark[p] = 1;
            queue[tail++] = p;
        }
    }
    while (head < tail) {
        int64_t p = queue[head++];
        int y = (int)(p / W), x = (int)(p % W);
        for (int dy = -1; dy <= 1; dy++) {
            for (int dx = -1; dx <= 1; dx++) {
                int yy = y + dy, xx = x + dx;
                if (yy < 0 || yy >= H || xx < 0 || xx >= W)
                    continue;
                int64_t q = (int64_t)yy * W + xx;
                if (b[q] && !mark[q]) {
                    mark[q] = 1;
                    queue[tail++] = q;
                }
            }
        }
    }
    oracle_near(mark, H, W, out);
    free(mark);
    free(queue);
    return ORC_OK;
}

/* interior a = !N!a */
int oracle_interior(const uint8_t *a, int H, int W, uint8_t *out)
{
    int64_t n = (int64_t)H * W;
    uint8_t *t = (uint8_t *)malloc((size_t)(n ? n : 1));
    if (!t)
        return ORC_ENOMEM;
    oracle_not(a, n, t);
    oracle_near(t, H, W, out);
    oracle_not(out, n, out);
    free(t);
    return ORC_OK;
}

/* surrounded(a,b) = a & !rho(!a & !b)[!b] */
int oracle_surrounded(const uint8_t *a, const uint8_t *b, int H, int W, uint8_t *out)
{
    int64_t n = (int64_t)H * W;
    size_t sz = (size_t)(n ? n : 1);
    uint8_t *na = (uint8_t *)malloc(sz), *nb = (uint8_t *)malloc(sz);
    uint8_t *esc = (uint8_t *)malloc(sz), *r = (uint8_t *)malloc(sz);
    int rc = ORC_ENOMEM;
    if (na && nb && esc && r) {
        oracle_not(a, n, na);
        oracle_not(b, n, nb);
        oracle_and(na, nb, n, esc);
        rc = oracle_reach(esc, nb, H, W, r);
        if (rc == ORC_OK) {
            oracle_not(r, n, r);
            oracle_and(a, r, n, out);
        }
    }
    free(na);
    free(nb);
    free(esc);
    free(r);
    return rc;
}

/* grow(a,b) = a | (b & rho a[b]) */
int oracle_grow(const uint8_t *a, const uint8_t *b, int H, int W, uint8_t *out)
{
    int64_t n = (int64_t)H * W;
    uint8_t *r = (uint8_t *)malloc((size_t)(n ? n : 1));
    if (!r)
        return ORC_ENOMEM;
    int rc = oracle_reach(a, b, H, W, r);
    if (rc == ORC_OK) {
        oracle_and(b, r, n, r);
        oracle_or(a, r, n, out);
    }
    free(r);
    return rc;
}

/* Connected-component labelling of a (8-connectivity), raster scan with a
 * breadth-first flood from each unlabelled pixel.  A component's label is the
 * row-major linear index y*W+x of its first pixel in raster order, i.e. its
 * smallest index; background pixels get -1. */
int oracle_ccl(const uint8_t *a, int H, int W, int32_t *lab)
{
    int64_t n = (int64_t)H * W;
    if (n == 0)
        return ORC_OK;
    int64_t *queue = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!queue)
        return ORC_ENOMEM;
    for (int64_t p = 0; p < n; p++)
        lab[p] = -1;
    for (int64_t s = 0; s < n; s++) {
        if (!a[s] || lab[s] >= 0)
            continue;
        int64_t head = 0, tail = 0;
        lab[s] = (int32_t)s;
        queue[tail++] = s;
        while (head < tail) {
            int64_t p = queue[head++];
            int y = (int)(p / W), x = (int)(p % W);
            for (int dy = -1; dy <= 1; dy++) {
                for (int dx = -1; dx <= 1; dx++) {
                    int yy = y + dy, xx = x + dx;
                    if (yy < 0 || yy >= H || xx < 0 || xx >= W)
                        continue;
                    int64_t q = (int64_t)yy * W + xx;
                    if (a[q] && lab[q] < 0) {
                        lab[q] = (int32_t)s;
                        queue[tail++] = q;
                    }
                }
            }
        }
    }
    free(queue);
    return ORC_OK;
}

/* Labels of the paper's own labelling algorithm once it has terminated
 * (Sect. 3, Alg. CCL): every pixel of a component carries the largest
 * coordinate pair of the component in lexicographic order, null elsewhere.
 * Coordinates are read as (row, column), so the order is the row-major
 * linear order and the label is written as the linear index y*W+x of the
 * component's last pixel in raster order; background pixels get -1.
 * Plain definition: a flood from each unlabelled pixel in reverse raster
 * order, so the flood's first pixel is the component's largest. */
int oracle_ccl_max(const uint8_t *a, int H, int W, int32_t *lab)
{
    int64_t n = (int64_t)H * W;
    if (n == 0)
        return ORC_OK;
    int64_t *queue = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!queue)
        return ORC_ENOMEM;
    for (int64_t p = 0; p < n; p++)
        lab[p] = -1;
    for (int64_t s = n - 1; s >= 0; s--) {
        if (!a[s] || lab[s] >= 0)
            continue;
        int64_t head = 0, tail = 0;
        lab[s] = (int32_t)s;
        queue[tail++] = s;
        while (head < tail) {
            int64_t p = queue[head++];
            int y = (int)(p / W), x = (int)(p % W);
            for (int dy = -1; dy <= 1; dy++) {
                for (int dx = -1; dx <= 1; dx++) {
                    int yy = y + dy, xx = x + dx;
                    if (yy < 0 || yy >= H || xx < 0 || xx >= W)
                        continue;
                    int64_t q = (int64_t)yy * W + xx;
                    if (a[q] && lab[q] < 0) {
                        lab[q] = lab[s]; /* the flood's first pixel */
                        queue[tail++] = q;
                    }
                }
            }
        }
    }
    free(queue);
    return ORC_OK;
}

/* ---- The paper's labelling algorithm, step by step (Sect. 3, Alg. CCL) ----
 *
 * Labels are coordinate pairs (i, j) = (row, column), compared
 * lexicographically; null (a background pixel) is below every pair.
 *   initialization: a pixel of `start` is labelled with its own coordinates.
 *   mainIteration:  a pixel of `start` holding (i', j') takes the largest
 *                   label in the Moore neighbourhood of (i', j') (that pixel
 *                   included) of the input labels; pointer jumping.
 *   reconnect:      a pixel of `start` at (i, j) holding (i', j') compares
 *                   the largest label (a, b) around (i, j) with the label
 *                   (c, d) stored at (i', j'); if (a, b) is larger it is
 *                   written at (i', j').  The paper asks for an atomic write
 *                   there without saying which of several writers wins;
 *                   read as an atomic maximum over the writers, into a copy
 *                   of the input labels (so the step reads only its input).
 *   termination:    done when no pixel of `start` has a neighbour of
 *                   `start` with a different label.
 * Schedule: after initialization, rounds of k main iterations, one
 * reconnect, then the termination check, until it reports done (Fig.
 * cc-movie: reconnect every 8 main iterations, termination after 24).
 * *iterations receives the number of main iterations.  At most max_rounds
 * rounds; if the check still fails, returns -6. */
typedef struct {
    int32_t i, j; /* i = -1: null */
} PjLabel;

static int pj_greater(PjLabel x, PjLabel y)
{
    return x.i > y.i || (x.i == y.i && x.j > y.j);
}

static PjLabel pj_max_neighbour(const PjLabel *in, int H, int W, int i, int j)
{
    PjLabel m = {-1, -1};
    for (int di = -1; di <= 1; di++) {
        for (int dj = -1; dj <= 1; dj++) {
            int ii = i + di, jj = j + dj;
            if (ii < 0 || ii >= H || jj < 0 || jj >= W)
                continue;
            PjLabel v = in[(int64_t)ii * W + jj];
            if (pj_greater(v, m))
                m = v;
        }
    }
    return m;
}

int oracle_ccl_pj(const uint8_t *start, int H, int W, int k, int max_rounds, int32_t *lab,
                  int64_t *iterations)
{
    int64_t n = (int64_t)H * W;
    *iterations = 0;
    if (k < 1 || max_rounds < 1)
        return ORC_EINVAL;
    if (n == 0)
        return ORC_OK;
    PjLabel *A = (PjLabel *)malloc((size_t)n * sizeof(PjLabel));
    PjLabel *B = (PjLabel *)malloc((size_t)n * sizeof(PjLabel));
    if (!A || !B) {
        free(A);
        free(B);
        return ORC_ENOMEM;
    }
    /* initialization */
    for (int i = 0; i < H; i++) {
        for (int j = 0; j < W; j++) {
            PjLabel v = {-1, -1};
            if (start[(int64_t)i * W + j]) {
                v.i = i;
                v.j = j;
            }
            A[(int64_t)i * W + j] = v;
            B[(int64_t)i * W + j] = v;
        }
    }
    int done = 0;
    for (int round = 0; round < max_rounds && !done; round++) {
        /* k main iterations, input A -> output B, then swap */
        for (int it = 0; it < k; it++) {
            for (int i = 0; i < H; i++) {
                for (int j = 0; j < W; j++) {
                    int64_t p = (int64_t)i * W + j;
                    if (!start[p])
                        continue;
                    PjLabel ij = A[p];
                    B[p] = pj_max_neighbour(A, H, W, ij.i, ij.j);
                }
            }
            PjLabel *t = A;
            A = B;
            B = t;
            (*iterations)++;
        }
        /* reconnect: input A, output B = copy of A raised by atomic maxima */
        memcpy(B, A, (size_t)n * sizeof(PjLabel));
        for (int i = 0; i < H; i++) {
            for (int j = 0; j < W; j++) {
                int64_t p = (int64_t)i * W + j;
                if (!start[p])
                    continue;
                PjLabel ij = A[p];
                PjLabel ab = pj_max_neighbour(A, H, W, i, j);
                int64_t q = (int64_t)ij.i * W + ij.j;
                PjLabel cd = A[q];
                if (pj_greater(ab, cd) && pj_greater(ab, B[q]))
                    B[q] = ab;
            }
        }
        PjLabel *t = A;
        A = B;
        B = t;
        /* termination check on the labels after the reconnect */
        done = 1;
        for (int i = 0; i < H && done; i++) {
            for (int j = 0; j < W && done; j++) {
                int64_t p = (int64_t)i * W + j;
                if (!start[p])
                    continue;
                for (int di = -1; di <= 1 && done; di++) {
                    for (int dj = -1; dj <= 1; dj++) {
                        int ii = i + di, jj = j + dj;
                        if (ii < 0 || ii >= H || jj < 0 || jj >= W)
                            continue;
                        int64_t q = (int64_t)ii * W + jj;
                        if (start[q] && (A[q].i != A[p].i || A[q].j != A[p].j)) {
                            done = 0;
                            break;
                        }
                    }
                }
            }
        }
    }
    for (int64_t p = 0; p < n; p++)
        lab[p] = A[p].i < 0 ? -1 : (int32_t)((int64_t)A[p].i * W + A[p].j);
    free(A);
    free(B);
    return done ? ORC_OK : -6;
}

/* ---- Volumes (D x H x W, slice-major) ----
 * The logic on 3-D images (the paper's tool is restricted to 2-D; its
 * limitation named in Sect. 1, Sect. 3 and Sect. 5): the Moore neighbourhood
 * becomes the 26 voxels sharing a face, an edge or a vertex, the voxel
 * itself included; paths step between such neighbours.  With D = 1 every
 * function equals its 2-D counterpart. */

/* N a over voxels: (z,y,x) is set iff a voxel of a lies in the 3x3x3 block
 * centred on it, counting only voxels inside the volume. */
void oracle_near3(const uint8_t *a, int D, int H, int W, uint8_t *out)
{
    for (int z = 0; z < D; z++) {
        for (int y = 0; y < H; y++) {
            for (int x = 0; x < W; x++) {
                int v = 0;
                for (int dz = -1; !v && dz <= 1; dz++) {
                    for (int dy = -1; !v && dy <= 1; dy++) {
                        for (int dx = -1; dx <= 1; dx++) {
                            int zz = z + dz, yy = y + dy, xx = x + dx;
                            if (zz < 0 || zz >= D || yy < 0 || yy >= H || xx < 0 || xx >= W)
                                continue;
                            if (a[((int64_t)zz * H + yy) * W + xx]) {
                                v = 1;
                                break;
                            }
                        }
                    }
                }
                out[((int64_t)z * H + y) * W + x] = (uint8_t)v;
            }
        }
    }
}

/* Flood from every voxel of a through 26-neighbours that satisfy b; marks
 * every flooded voxel in mark (caller-zeroed). */
static int flood3(const uint8_t *a, const uint8_t *b, int D, int H, int W, uint8_t *mark)
{
    int64_t n = (int64_t)D * H * W;
    int64_t *queue = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
    if (!queue)
        return ORC_ENOMEM;
    int64_t head = 0, tail = 0;
    for (int64_t p = 0; p < n; p++) {
        if (!a[p])
            continue;
        mark[p] = 1;
        queue[tail++] = p;
    }
    while (head < tail) {
        int64_t p = queue[head++];
        int z = (int)(p / ((int64_t)H * W)), y = (int)(p / W % H), x = (int)(p % W);
        for (int dz = -1; dz <= 1; dz++) {
            for (int dy = -1; dy <= 1; dy++) {
                for (int dx = -1; dx <= 1; dx++) {
                    int zz = z + dz, yy = y + dy, xx = x + dx;
                    if (zz < 0 || zz >= D || yy < 0 || yy >= H || xx < 0 || xx >= W)
                        continue;
                    int64_t q = ((int64_t)zz * H + yy) * W + xx;
                    if (!mark[q] && b[q]) {
                        mark[q] = 1;
                        queue[tail++] = q;
                    }
                }
            }
        }
    }
    free(queue);
    return ORC_OK;
}

/* rho a[b] over voxels: flood from a through b, then one dilation. */
int oracle_reach3(const uint8_t *a, const uint8_t *b, int D, int H, int W, uint8_t *out)
{
    int64_t n = (int64_t)D * H * W;
    uint8_t *mark = (uint8_t *)calloc((size_t)(n ? n : 1), 1);
    if (!mark)
        return ORC_ENOMEM;
    int rc = flood3(a, b, D, H, W, mark);
    if (rc == ORC_OK)
        oracle_near3(mark, D, H, W, out);
    free(mark);
    return rc;
}

/* 26-connected labels of a volume: a flood from each unlabelled voxel in
 * raster order; label = the flood's first voxel = the smallest linear index
 * (z*H + y)*W + x of the component; -1 for background. */
int oracle_ccl3(const uint8_t *a, int D, int H, int W, int32_t *lab)
{
    int64_t n = (int64_t)D * H * W;
    if (n == 0)
        return ORC_OK;
    int64_t *queue = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!queue)
        return ORC_ENOMEM;
    for (int64_t p = 0; p < n; p++)
        lab[p] = -1;
    for (int64_t s = 0; s < n; s++) {
        if (!a[s] || lab[s] >= 0)
            continue;
        int64_t head = 0, tail = 0;
        lab[s] = (int32_t)s;
        queue[tail++] = s;
        while (head < tail) {
            int64_t p = queue[head++];
            int z = (int)(p / ((int64_t)H * W)), y = (int)(p / W % H), x = (int)(p % W);
            for (int dz = -1; dz <= 1; dz++) {
                for (int dy = -1; dy <= 1; dy++) {
                    for (int dx = -1; dx <= 1; dx++) {
                        int zz = z + dz, yy = y + dy, xx = x + dx;
                        if (zz < 0 || zz >= D || yy < 0 || yy >= H || xx < 0 || xx >= W)
                            continue;
                        int64_t q = ((int64_t)zz * H + yy) * W + xx;
                        if (a[q] && lab[q] < 0) {
                            lab[q] = lab[s]; /* the flood's first voxel */
                            queue[tail++] = q;
                        }
                    }
                }
            }
        }
    }
    free(queue);
    return ORC_OK;
}

static float pixel_value(const void *img, int dtype, int64_t idx)
{
    if (dtype == DT_U8)
        return (float)((const uint8_t *)img)[idx];
    if (dtype == DT_U16)
        return (float)((const uint16_t *)img)[idx]; /* exact: 16 bits fit the float32 mantissa */
    return ((const float *)img)[idx];
}

static int cmp_float(const void *pa, const void *pb)
{
    float a = *(const float *)pa, b = *(const float *)pb;
    return (a < b) ? -1 : (a > b) ? 1 : 0;
}

/* k-th smallest value of channel c, k = clamp(ceil(q*n) - 1, 0, n - 1). */
int oracle_percentile(const void *img, int dtype, int C, int H, int W, int c, double q,
                      float *result)
{
    if (c < 0 || c >= C)
        return ORC_EINVAL;
    int64_t n = (int64_t)H * W;
    if (n == 0) {
        *result = 0.0f;
        return ORC_OK;
    }
    float *v = (float *)malloc((size_t)n * sizeof(float));
    if (!v)
        return ORC_ENOMEM;
    for (int64_t i = 0; i < n; i++)
        v[i] = pixel_value(img, dtype, (int64_t)c * n + i);
    qsort(v, (size_t)n, sizeof(float), cmp_float);
    double kk = ceil(q * (double)n) - 1.0;
    int64_t k = kk < 0.0 ? 0 : (kk > (double)(n - 1) ? n - 1 : (int64_t)kk);
    *result = v[k];
    free(v);
    return ORC_OK;
}

#define CMP_GT 0
#define CMP_LT 1
#define CMP_GE 2
#define CMP_LE 3

/* Threshold atom: out = (float32(img[c]) OP t) pixel-wise, in float32. */
int oracle_threshold(const void *img, int dtype, int C, int H, int W, int c, int op, float t,
                     uint8_t *out)
{
    if (c < 0 || c >= C || op < 0 || op > 3)
        return ORC_EINVAL;
    int64_t n = (int64_t)H * W;
    for (int64_t i = 0; i < n; i++) {
        float v = pixel_value(img, dtype, (int64_t)c * n + i);
        int r;
        switch (op) {
        case CMP_GT: r = v > t; break;
        case CMP_LT: r = v < t; break;
        case CMP_GE: r = v >= t; break;
        default: r = v <= t; break;
        }
        out[i] = (uint8_t)(r ? 1 : 0);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Formula language (ImgQL subset, paper Sect. 3 Syntax)               */
/*                                                                     */
/*   program := { 'let' NAME [ '(' NAME {',' NAME} ')' ] '=' expr      */
/*              | 'output' STRING expr } (';' optional)                */
/*   expr := and { '|' and }     and := un { '&' un }                  */
/*   un := '!' un | prim                                               */
/*   prim := 'true' | 'false' | '(' expr ')'                           */
/*         | 'intensity' '(' 'img' [',' INT] ')' CMP scalar            */
/*         | NAME [ '(' expr {',' expr} ')' ]                          */
/*   CMP := '>.' | '<.' | '>=.' | '<=.'                                */
/*   scalar := ['-'] NUMBER | 'percentile' '(' 'img' ',' INT ',' NUMBER ')' */
/*   built-ins: near(e) N(e) interior(e) reach(a,b) surrounded(a,b)    */
/*              grow(a,b) touch(a,b); comments run from '//' to end of */
/*              line.                                                  */
/*   Arithmetic atoms (Sect. 3: the tool's built-in arithmetic):       */
/*   prim := num CMP num    (any atom that is not the form above)      */
/*   num := term { ('+' | '-') term }   term := fac { ('*' | '/') fac } */
/*   fac := '-' fac | NUMBER | 'intensity' '(' 'img' [',' INT] ')'      */
/*        | 'percentile' '(' 'img' ',' INT ',' NUMBER ')'               */
/*        | 'abs' '(' num ')' | ('min' | 'max') '(' num ',' num ')'     */
/*        | '(' num ')'                                                 */
/* ------------------------------------------------------------------ */

enum {
    K_TRUE, K_FALSE, K_ATOM, K_NOT, K_AND, K_OR, K_NEAR, K_INTERIOR,
    K_REACH, K_SURR, K_GROW, K_GLOBAL, K_PARAM, K_CALL, K_TOUCH,
    K_ARITH, /* atom a CMP b over numeric expressions a, b */
    /* numeric expression nodes (values per pixel, float32) */
    K_N_CONST, K_N_CHAN, K_N_PCT, K_N_NEG, K_N_ABS, K_N_ADD, K_N_SUB, K_N_MUL, K_N_DIV,
    K_N_MIN, K_N_MAX
};

typedef struct Node {
    int kind;
    struct Node *a, *b;
    struct Node **args;
    int nargs;
    int ref;          /* K_GLOBAL / K_CALL: definition index; K_PARAM: param index */
    int chan, cmp;    /* K_ATOM */
    int use_pct;      /* threshold is a percentile */
    float thr;
    int pchan;
    double pq;
    struct Node *next_alloc;
} Node;

typedef struct Def {
    char name[64];
    int nparams;
    char params[16][64];
    Node *body;
    uint8_t *value;
    int64_t refs_left;
    int pinned;
    int evaluated;
} Def;

typedef struct Stmt {
    int is_output;
    int def;         /* let: definition index */
    Node *expr;      /* output expression */
} Stmt;

typedef struct Prog {
    Def *defs;
    int ndefs, capdefs;
    Stmt *stmts;
    int nstmts, capstmts;
    int noutputs;
    Node *all_nodes;
} Prog;

typedef struct Parser {
    const char *src;
    size_t pos;
    int line, col;
    char *err;
    int errlen;
    int failed;
    Prog *prog;
    Def *cur_macro;  /* macro whose body is being parsed, or NULL */
} Parser;

static void perr(Parser *P, const char *msg)
{
    if (P->failed)
        return;
    P->failed = 1;
    if (P->err && P->errlen > 0)
        snprintf(P->err, (size_t)P->errlen, "line %d col %d: %s", P->line, P->col, msg);
}

static void adv(Parser *P)
{
    if (P->src[P->pos] == '\n') {
        P->line++;
        P->col = 1;
    } else {
        P->col++;
    }
    P->pos++;
}

static void skip_ws(Parser *P)
{
    for (;;) {
        char c = P->src[P->pos];
        if (c == ' ' || c == '\t' || c == '\r' || c == '\n' || c == ';') {
            adv(P);
        } else if (c == '/' && P->src[P->pos + 1] == '/') {
            while (P->src[P->pos] && P->src[P->pos] != '\n')
                adv(P);
        } else {
            return;
        }
    }
}

static int peek_char(Parser *P)
{
    skip_ws(P);
    return (unsigned char)P->src[P->pos];
}

static int accept(Parser *P, const char *s)
{
    skip_ws(P);
    size_t n = strlen(s);
    if (strncmp(P->src + P->pos, s, n) == 0) {
        for (size_t i = 0; i < n; i++)
            adv(P);
        return 1;
    }
    return 0;
}

static void expect(Parser *P, const char *s)
{
    if (!accept(P, s)) {
        char msg[96];
        snprintf(msg, sizeof msg, "expected '%s'", s);
        perr(P, msg);
    }
}

static int read_ident(Parser *P, char *out, size_t outlen)
{
    skip_ws(P);
    const char *s = P->src + P->pos;
    if (!(isalpha((unsigned char)s[0]) || s[0] == '_'))
        return 0;
    size_t n = 0;
    while (isalnum((unsigned char)s[n]) || s[n] == '_')
        n++;
    if (n >= outlen) {
        perr(P, "identifier too long");
        return 0;
    }
    memcpy(out, s, n);
    out[n] = 0;
    for (size_t i = 0; i < n; i++)
        adv(P);
    return 1;
}

static int read_number(Parser *P, double *v)
{
    skip_ws(P);
    const char *s = P->src + P->pos;
    if (!(isdigit((unsigned char)s[0]) || (s[0] == '.' && isdigit((unsigned char)s[1]))))
        return 0;
    char *end = NULL;
    *v = strtod(s, &end);
    size_t n = (size_t)(end - s);
    for (size_t i = 0; i < n; i++)
        adv(P);
    return 1;
}

static int read_int(Parser *P, int *v)
{
    skip_ws(P);
    const char *s = P->src + P->pos;
    if (!isdigit((unsigned char)s[0]))
        return 0;
    long x = 0;
    size_t n = 0;
    while (isdigit((unsigned char)s[n])) {
        x = x * 10 + (s[n] - '0');
        if (x > 1000000)
            break;
        n++;
    }
    for (size_t i = 0; i < n; i++)
        adv(P);
    *v = (int)x;
    return 1;
}

static Node *new_node(Parser *P, int kind)
{
    Node *n = (Node *)calloc(1, sizeof(Node));
    if (!n) {
        perr(P, "out of memory");
        return NULL;
    }
    n->kind = kind;
    n->next_alloc = P->prog->all_nodes;
    P->prog->all_nodes = n;
    return n;
}

static int find_def(Prog *G, const char *name)
{
    for (int i = G->ndefs - 1; i >= 0; i--)
        if (strcmp(G->defs[i].name, name) == 0)
            return i;
    return -1;
}

static int is_builtin(const char *s)
{
    static const char *names[] = {"let", "output", "true", "false", "intensity", "percentile",
                                  "img", "near", "N", "interior", "reach", "surrounded",
                                  "grow", "touch", "abs", "min", "max", NULL};
    for (int i = 0; names[i]; i++)
        if (strcmp(s, names[i]) == 0)
            return 1;
    return 0;
}

static Node *parse_expr(Parser *P);

static void parse_img_channel(Parser *P, int *chan, int allow_default)
{
    char id[64];
    if (!read_ident(P, id, sizeof id) || strcmp(id, "img") != 0) {
        perr(P, "expected 'img'");
        return;
    }
    *chan = 0;
    if (accept(P, ",")) {
        if (!read_int(P, chan))
            perr(P, "expected channel index");
    } else if (!allow_default) {
        perr(P, "expected ','");
    }
}

/* ---- arithmetic atoms ----
 * Numeric expressions are parsed speculatively: where the text at this point
 * is a numeric expression followed by a comparison, it is an arithmetic
 * atom; otherwise the parser backs up and reads a Boolean expression.  A
 * numeric parse fails quietly (NULL) on anything that is not numeric. */
static int peek_cmp(Parser *P)
{
    skip_ws(P);
    const char *t = P->src + P->pos;
    return strncmp(t, ">=.", 3) == 0 || strncmp(t, "<=.", 3) == 0 || strncmp(t, ">.", 2) == 0 ||
           strncmp(t, "<.", 2) == 0;
}

static Node *parse_num(Parser *P);

static Node *num_node(Parser *P, int kind, Node *a, Node *b)
{
    Node *n = new_node(P, kind);
    if (n) {
        n->a = a;
        n->b = b;
    }
    return n;
}

static Node *parse_num_factor(Parser *P)
{
    if (P->failed)
        return NULL;
    if (accept(P, "-")) {
        Node *a = parse_num_factor(P);
        return a ? num_node(P, K_N_NEG, a, NULL) : NULL;
    }
    if (accept(P, "(")) {
        Node *a = parse_num(P);
        if (!a || !accept(P, ")"))
            return NULL;
        return a;
    }
    double v;
    if (read_number(P, &v)) {
        Node *n = new_node(P, K_N_CONST);
        if (n)
            n->thr = (float)v; /* read as double, rounded once to float32 */
        return n;
    }
    char id[64];
    if (!read_ident(P, id, sizeof id))
        return NULL;
    if (strcmp(id, "intensity") == 0) {
        Node *n = new_node(P, K_N_CHAN);
        if (!n || !accept(P, "("))
            return NULL;
        parse_img_channel(P, &n->chan, 1);
        return (!P->failed && accept(P, ")")) ? n : NULL;
    }
    if (strcmp(id, "percentile") == 0) {
        Node *n = new_node(P, K_N_PCT);
        if (!n || !accept(P, "("))
            return NULL;
        parse_img_channel(P, &n->pchan, 0);
        if (P->failed || !accept(P, ",") || !read_number(P, &n->pq) || !accept(P, ")"))
            return NULL;
        return n;
    }
    if (strcmp(id, "abs") == 0) {
        if (!accept(P, "("))
            return NULL;
        Node *a = parse_num(P);
        if (!a || !accept(P, ")"))
            return NULL;
        return num_node(P, K_N_ABS, a, NULL);
    }
    if (strcmp(id, "min") == 0 || strcmp(id, "max") == 0) {
        int kind = id[1] == 'i' ? K_N_MIN : K_N_MAX;
        if (!accept(P, "("))
            return NULL;
        Node *a = parse_num(P);
        if (!a || !accept(P, ","))
            return NULL;
        Node *b = parse_num(P);
        if (!b || !accept(P, ")"))
            return NULL;
        return num_node(P, kind, a, b);
    }
    return NULL;
}

static Node *parse_num_term(Parser *P)
{
    Node *l = parse_num_factor(P);
    while (l) {
        int kind;
        if (accept(P, "*"))
            kind = K_N_MUL;
        else if (accept(P, "/"))
            kind = K_N_DIV;
        else
            break;
        Node *r = parse_num_factor(P);
        l = r ? num_node(P, kind, l, r) : NULL;
    }
    return l;
}

static Node *parse_num(Parser *P)
{
    Node *l = parse_num_term(P);
    while (l) {
        int kind;
        if (accept(P, "+"))
            kind = K_N_ADD;
        else if (accept(P, "-"))
            kind = K_N_SUB;
        else
            break;
        Node *r = parse_num_term(P);
        l = r ? num_node(P, kind, l, r) : NULL;
    }
    return l;
}

/* An arithmetic atom at the current position, or NULL (position unchanged)
 * when the text there is not a numeric expression followed by a comparison.
 * The paper's plain atom, intensity(img[, c]) CMP constant-or-percentile, is
 * returned as K_ATOM; every other comparison as K_ARITH. */
static Node *try_parse_arith_atom(Parser *P)
{
    size_t pos = P->pos;
    int line = P->line, col = P->col;
    Node *lhs = parse_num(P);
    if (P->failed)
        return NULL;
    if (!lhs || !peek_cmp(P)) {
        P->pos = pos;
        P->line = line;
        P->col = col;
        return NULL;
    }
    int cmp;
    if (accept(P, ">=."))
        cmp = CMP_GE;
    else if (accept(P, "<=."))
        cmp = CMP_LE;
    else if (accept(P, ">."))
        cmp = CMP_GT;
    else {
        accept(P, "<.");
        cmp = CMP_LT;
    }
    Node *rhs = parse_num(P);
    if (!rhs) {
        perr(P, "expected a numeric expression after the comparison");
        return NULL;
    }
    int rconst = rhs->kind == K_N_CONST ||
                 (rhs->kind == K_N_NEG && rhs->a->kind == K_N_CONST);
    if (lhs->kind == K_N_CHAN && (rconst || rhs->kind == K_N_PCT)) {
        Node *n = new_node(P, K_ATOM);
        if (!n)
            return NULL;
        n->chan = lhs->chan;
        n->cmp = cmp;
        if (rhs->kind == K_N_PCT) {
            n->use_pct = 1;
            n->pchan = rhs->pchan;
            n->pq = rhs->pq;
        } else {
            n->thr = rhs->kind == K_N_CONST ? rhs->thr : -rhs->a->thr;
        }
        return n;
    }
    Node *n = new_node(P, K_ARITH);
    if (n) {
        n->a = lhs;
        n->b = rhs;
        n->cmp = cmp;
    }
    return n;
}

static Node *parse_call_args(Parser *P, Node *n, int want)
{
    expect(P, "(");
    n->a = parse_expr(P);
    if (want == 2) {
        expect(P, ",");
        n->b = parse_expr(P);
    }
    expect(P, ")");
    return n;
}

static Node *parse_prim(Parser *P)
{
    if (P->failed)
        return NULL;
    Node *at = try_parse_arith_atom(P);
    if (at || P->failed)
        return at;
    if (accept(P, "(")) {
        Node *e = parse_expr(P);
        expect(P, ")");
        return e;
    }
    char id[64];
    if (!read_ident(P, id, sizeof id)) {
        perr(P, "expected an expression");
        return NULL;
    }
    if (strcmp(id, "true") == 0)
        return new_node(P, K_TRUE);
    if (strcmp(id, "false") == 0)
        return new_node(P, K_FALSE);
    if (strcmp(id, "intensity") == 0 || strcmp(id, "percentile") == 0 || strcmp(id, "abs") == 0 ||
        strcmp(id, "min") == 0 || strcmp(id, "max") == 0) {
        perr(P, "expected a comparison '>.', '<.', '>=.' or '<=.' after a numeric expression");
        return NULL;
    }
    if (strcmp(id, "near") == 0 || strcmp(id, "N") == 0)
        return parse_call_args(P, new_node(P, K_NEAR), 1);
    if (strcmp(id, "interior") == 0)
        return parse_call_args(P, new_node(P, K_INTERIOR), 1);
    if (strcmp(id, "reach") == 0)
        return parse_call_args(P, new_node(P, K_REACH), 2);
    if (strcmp(id, "surrounded") == 0)
        return parse_call_args(P, new_node(P, K_SURR), 2);
    if (strcmp(id, "grow") == 0)
        return parse_call_args(P, new_node(P, K_GROW), 2);
    if (strcmp(id, "touch") == 0)
        return parse_call_args(P, new_node(P, K_TOUCH), 2);
    if (is_builtin(id)) {
        perr(P, "unexpected keyword");
        return NULL;
    }
    /* parameter of the macro being defined? */
    if (P->cur_macro) {
        for (int i = 0; i < P->cur_macro->nparams; i++) {
            if (strcmp(P->cur_macro->params[i], id) == 0) {
                Node *n = new_node(P, K_PARAM);
                if (n)
                    n->ref = i;
                return n;
            }
        }
    }
    int d = find_def(P->prog, id);
    if (d < 0) {
        char msg[128];
        snprintf(msg, sizeof msg, "undefined name '%s'", id);
        perr(P, msg);
        return NULL;
    }
    Def *D = &P->prog->defs[d];
    if (D->nparams > 0) {
        Node *n = new_node(P, K_CALL);
        if (!n)
            return NULL;
        n->ref = d;
        n->args = (Node **)calloc((size_t)D->nparams, sizeof(Node *));
        n->nargs = D->nparams;
        expect(P, "(");
        for (int i = 0; i < D->nparams && !P->failed; i++) {
            if (i > 0)
                expect(P, ",");
            n->args[i] = parse_expr(P);
        }
        expect(P, ")");
        return n;
    }
    Node *n = new_node(P, K_GLOBAL);
    if (!n)
        return NULL;
    n->ref = d;
    if (P->cur_macro)
        D->pinned = 1;
    else
        D->refs_left++;
    return n;
}

static Node *parse_unary(Parser *P)
{
    if (P->failed)
        return NULL;
    if (accept(P, "!")) {
        Node *n = new_node(P, K_NOT);
        if (n)
            n->a = parse_unary(P);
        return n;
    }
    return parse_prim(P);
}

static Node *parse_and(Parser *P)
{
    Node *l = parse_unary(P);
    while (!P->failed && accept(P, "&")) {
        Node *n = new_node(P, K_AND);
        if (!n)
            return NULL;
        n->a = l;
        n->b = parse_unary(P);
        l = n;
    }
    return l;
}

static Node *parse_expr(Parser *P)
{
    Node *l = parse_and(P);
    while (!P->failed && accept(P, "|")) {
        Node *n = new_node(P, K_OR);
        if (!n)
            return NULL;
        n->a = l;
        n->b = parse_and(P);
        l = n;
    }
    return l;
}

static int add_stmt(Prog *G, Stmt s)
{
    if (G->nstmts == G->capstmts) {
        int cap = G->capstmts ? 2 * G->capstmts : 64;
        Stmt *ns = (Stmt *)realloc(G->stmts, (size_t)cap * sizeof(Stmt));
        if (!ns)
            return 0;
        G->stmts = ns;
        G->capstmts = cap;
    }
    G->stmts[G->nstmts++] = s;
    return 1;
}

static int add_def(Prog *G)
{
    if (G->ndefs == G->capdefs) {
        int cap = G->capdefs ? 2 * G->capdefs : 64;
        Def *nd = (Def *)realloc(G->defs, (size_t)cap * sizeof(Def));
        if (!nd)
            return -1;
        G->defs = nd;
        G->capdefs = cap;
    }
    memset(&G->defs[G->ndefs], 0, sizeof(Def));
    return G->ndefs++;
}

static void free_prog(Prog *G)
{
    Node *n = G->all_nodes;
    while (n) {
        Node *nx = n->next_alloc;
        free(n->args);
        free(n);
        n = nx;
    }
    for (int i = 0; i < G->ndefs; i++)
        free(G->defs[i].value);
    free(G->defs);
    free(G->stmts);
    memset(G, 0, sizeof *G);
}

static int parse_program(const char *src, Prog *G, char *err, int errlen)
{
    Parser P;
    memset(&P, 0, sizeof P);
    P.src = src;
    P.line = 1;
    P.col = 1;
    P.err = err;
    P.errlen = errlen;
    P.prog = G;
    while (!P.failed && peek_char(&P) != 0) {
        char kw[64];
        if (!read_ident(&P, kw, sizeof kw)) {
            perr(&P, "expected 'let' or 'output'");
            break;
        }
        if (strcmp(kw, "let") == 0) {
            char name[64];
            if (!read_ident(&P, name, sizeof name)) {
                perr(&P, "expected a name after 'let'");
                break;
            }
            if (is_builtin(name)) {
                perr(&P, "cannot redefine a built-in name");
                break;
            }
            Def tmp;
            memset(&tmp, 0, sizeof tmp);
            snprintf(tmp.name, sizeof tmp.name, "%s", name);
            if (accept(&P, "(")) {
                do {
                    if (tmp.nparams >= 16) {
                        perr(&P, "too many parameters");
                        break;
                    }
                    if (!read_ident(&P, tmp.params[tmp.nparams], sizeof tmp.params[0])) {
                        perr(&P, "expected a parameter name");
                        break;
                    }
                    tmp.nparams++;
                } while (accept(&P, ","));
                expect(&P, ")");
            }
            expect(&P, "=");
            if (P.failed)
                break;
            /* the body is parsed before the name is bound: no recursion */
            P.cur_macro = tmp.nparams > 0 ? &tmp : NULL;
            Node *body = parse_expr(&P);
            P.cur_macro = NULL;
            if (P.failed)
                break;
            int d = add_def(G);
            if (d < 0) {
                perr(&P, "out of memory");
                break;
            }
            tmp.body = body;
            G->defs[d] = tmp;
            Stmt s = {0, d, NULL};
            if (!add_stmt(G, s)) {
                perr(&P, "out of memory");
                break;
            }
        } else if (strcmp(kw, "output") == 0) {
            skip_ws(&P);
            if (P.src[P.pos] != '"') {
                perr(&P, "expected a quoted output name");
                break;
            }
            adv(&P);
            while (P.src[P.pos] && P.src[P.pos] != '"' && P.src[P.pos] != '\n')
                adv(&P);
            if (P.src[P.pos] != '"') {
                perr(&P, "unterminated string");
                break;
            }
            adv(&P);
            Node *e = parse_expr(&P);
            if (P.failed)
                break;
            Stmt s = {1, -1, e};
            if (!add_stmt(G, s)) {
                perr(&P, "out of memory");
                break;
            }
            G->noutputs++;
        } else {
            perr(&P, "expected 'let' or 'output'");
        }
    }
    return P.failed ? ORC_EPARSE : ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Evaluation                                                          */
/* ------------------------------------------------------------------ */

typedef struct Ctx {
    Prog *G;
    const void *img;
    int dtype, C, D, H, W; /* D slices of H x W (D = 1: a 2-D image) */
    int64_t n;
    char *err;
    int errlen;
    int rc;
} Ctx;

static uint8_t *alloc_mask(Ctx *X)
{
    uint8_t *m = (uint8_t *)malloc((size_t)(X->n ? X->n : 1));
    if (!m && X->rc == ORC_OK)
        X->rc = ORC_ENOMEM;
    return m;
}

/* Numeric expressions, pixel by pixel in float32: every operation rounds
 * once (IEEE single, round to nearest even; no fused multiply-add), min and
 * max keep the first operand unless the second compares below (above) it,
 * abs and unary minus act on the sign.  Percentile leaves are computed once
 * per evaluation of their atom (num_prepare). */
static int num_prepare(Ctx *X, Node *e)
{
    if (!e)
        return ORC_OK;
    if (e->kind == K_N_CHAN && (e->chan < 0 || e->chan >= X->C)) {
        X->rc = ORC_EINVAL;
        if (X->err && X->errlen > 0)
            snprintf(X->err, (size_t)X->errlen, "channel index out of range");
        return X->rc;
    }
    if (e->kind == K_N_PCT) {
        if (e->pchan < 0 || e->pchan >= X->C) {
            X->rc = ORC_EINVAL;
            if (X->err && X->errlen > 0)
                snprintf(X->err, (size_t)X->errlen, "channel index out of range");
            return X->rc;
        }
        int rc = oracle_percentile(X->img, X->dtype, X->C, X->D * X->H, X->W, e->pchan, e->pq, &e->thr);
        if (rc != ORC_OK)
            X->rc = rc;
        return rc;
    }
    int rc = num_prepare(X, e->a);
    return rc == ORC_OK ? num_prepare(X, e->b) : rc;
}

static float num_eval(Ctx *X, Node *e, int64_t i)
{
    float a, b;
    switch (e->kind) {
    case K_N_CONST:
    case K_N_PCT:
        return e->thr;
    case K_N_CHAN:
        return pixel_value(X->img, X->dtype, (int64_t)e->chan * X->n + i);
    case K_N_NEG:
        return -num_eval(X, e->a, i);
    case K_N_ABS:
        return fabsf(num_eval(X, e->a, i));
    default:
        break;
    }
    a = num_eval(X, e->a, i);
    b = num_eval(X, e->b, i);
    switch (e->kind) {
    case K_N_ADD: return a + b;
    case K_N_SUB: return a - b;
    case K_N_MUL: return a * b;
    case K_N_DIV: return a / b;
    case K_N_MIN: return b < a ? b : a;
    default: return b > a ? b : a; /* K_N_MAX */
    }
}

/* reach, surrounded and grow on a volume, by the same definitions as in 2-D:
 * surrounded(a,b) = a & !rho(!a & !b)[!b], grow(a,b) = a | (b & rho a[b]). */
static int reach_like3(Ctx *X, int kind, const uint8_t *a, const uint8_t *b, uint8_t *out)
{
    int64_t n = X->n;
    if (kind == K_REACH)
        return oracle_reach3(a, b, X->D, X->H, X->W, out);
    uint8_t *t = (uint8_t *)malloc((size_t)(n ? n : 1)), *u = (uint8_t *)malloc((size_t)(n ? n : 1));
    int rc = ORC_ENOMEM;
    if (t && u) {
        if (kind == K_GROW) {
            rc = oracle_reach3(a, b, X->D, X->H, X->W, t);
            if (rc == ORC_OK) {
                oracle_and(b, t, n, t);
                oracle_or(a, t, n, out);
            }
        } else {
            oracle_not(a, n, t);
            oracle_not(b, n, u);
            oracle_and(t, u, n, t); /* !a & !b */
            rc = oracle_reach3(t, u, X->D, X->H, X->W, out);
            if (rc == ORC_OK) {
                oracle_not(out, n, out);
                oracle_and(a, out, n, out);
            }
        }
    }
    free(t);
    free(u);
    return rc;
}

/* Evaluate e; params (may be NULL) are the masks bound to the parameters of the
 * macro whose body is being evaluated.  Returns a fresh mask owned by the
 * caller, or NULL on error. */
static uint8_t *eval(Ctx *X, Node *e, uint8_t **params)
{
    if (!e || X->rc != ORC_OK)
        return NULL;
    int64_t n = X->n;
    uint8_t *out = NULL, *a = NULL, *b = NULL;
    switch (e->kind) {
    case K_TRUE:
    case K_FALSE:
        out = alloc_mask(X);
        if (out)
            memset(out, e->kind == K_TRUE ? 1 : 0, (size_t)n);
        return out;
    case K_ATOM: {
        float t = e->thr;
        if (e->chan < 0 || e->chan >= X->C || (e->use_pct && (e->pchan < 0 || e->pchan >= X->C))) {
            X->rc = ORC_EINVAL;
            if (X->err && X->errlen > 0)
                snprintf(X->err, (size_t)X->errlen, "channel index out of range");
            return NULL;
        }
        if (e->use_pct) {
            int rc = oracle_percentile(X->img, X->dtype, X->C, X->D * X->H, X->W, e->pchan, e->pq, &t);
            if (rc != ORC_OK) {
                X->rc = rc;
                return NULL;
            }
        }
        out = alloc_mask(X);
        if (!out)
            return NULL;
        oracle_threshold(X->img, X->dtype, X->C, X->D * X->H, X->W, e->chan, e->cmp, t, out);
        return out;
    }
    case K_ARITH: {
        if (num_prepare(X, e->a) != ORC_OK || num_prepare(X, e->b) != ORC_OK)
            return NULL;
        out = alloc_mask(X);
        if (!out)
            return NULL;
        for (int64_t i = 0; i < n; i++) {
            float v = num_eval(X, e->a, i), t = num_eval(X, e->b, i);
            out[i] = (uint8_t)(e->cmp == CMP_GT ? v > t : e->cmp == CMP_LT ? v < t : e->cmp == CMP_GE ? v >= t : v <= t);
        }
        return out;
    }
    case K_TOUCH: /* touch(a, b) = a & rho b[a] */
        a = eval(X, e->a, params);
        b = eval(X, e->b, params);
        out = (a && b) ? alloc_mask(X) : NULL;
        if (out) {
            int rc = X->D == 1 ? oracle_reach(b, a, X->H, X->W, out) : oracle_reach3(b, a, X->D, X->H, X->W, out);
            if (rc == ORC_OK) {
                oracle_and(a, out, n, out);
            } else {
                X->rc = rc;
                free(out);
                out = NULL;
            }
        }
        free(a);
        free(b);
        return out;
    case K_NOT:
        a = eval(X, e->a, params);
        if (!a)
            return NULL;
        oracle_not(a, n, a);
        return a;
    case K_AND:
    case K_OR:
        a = eval(X, e->a, params);
        b = eval(X, e->b, params);
        if (a && b) {
            if (e->kind == K_AND)
                oracle_and(a, b, n, a);
            else
                oracle_or(a, b, n, a);
            free(b);
            return a;
        }
        free(a);
        free(b);
        return NULL;
    case K_NEAR:
    case K_INTERIOR:
        a = eval(X, e->a, params);
        if (!a)
            return NULL;
        out = alloc_mask(X);
        if (out && X->D > 1) { /* volumes: N over 26 neighbours, interior = !N! */
            if (e->kind == K_INTERIOR)
                oracle_not(a, n, a);
            oracle_near3(a, X->D, X->H, X->W, out);
            if (e->kind == K_INTERIOR)
                oracle_not(out, n, out);
        } else if (out) {
            if (e->kind == K_NEAR)
                oracle_near(a, X->H, X->W, out);
            else if (oracle_interior(a, X->H, X->W, out) != ORC_OK) {
                X->rc = ORC_ENOMEM;
                free(out);
                out = NULL;
            }
        }
        free(a);
        return out;
    case K_REACH:
    case K_SURR:
    case K_GROW: {
        int rc3;
        a = eval(X, e->a, params);
        b = eval(X, e->b, params);
        out = (a && b) ? alloc_mask(X) : NULL;
        if (out && X->D > 1) {
            rc3 = reach_like3(X, e->kind, a, b, out);
            if (rc3 != ORC_OK) {
                X->rc = rc3;
                free(out);
                out = NULL;
            }
        } else if (out) {
            int rc;
            if (e->kind == K_REACH)
                rc = oracle_reach(a, b, X->H, X->W, out);
            else if (e->kind == K_SURR)
                rc = oracle_surrounded(a, b, X->H, X->W, out);
            else
                rc = oracle_grow(a, b, X->H, X->W, out);
            if (rc != ORC_OK) {
                X->rc = rc;
                free(out);
                out = NULL;
            }
        }
        free(a);
        free(b);
        return out;
    }
    case K_PARAM:
        out = alloc_mask(X);
        if (out)
            memcpy(out, params[e->ref], (size_t)n);
        return out;
    case K_GLOBAL: {
        Def *D = &X->G->defs[e->ref];
        if (!D->evaluated || !D->value) {
            X->rc = ORC_EINVAL;
            if (X->err && X->errlen > 0)
                snprintf(X->err, (size_t)X->errlen, "internal: '%s' not evaluated", D->name);
            return NULL;
        }
        out = alloc_mask(X);
        if (out)
            memcpy(out, D->value, (size_t)n);
        /* a reference from top-level code is read exactly once */
        if (!params && !D->pinned && --D->refs_left == 0) {
            free(D->value);
            D->value = NULL;
        }
        return out;
    }
    case K_CALL: {
        Def *D = &X->G->defs[e->ref];
        uint8_t *argv[16] = {0};
        int ok = 1;
        for (int i = 0; i < e->nargs; i++) {
            argv[i] = eval(X, e->args[i], params);
            if (!argv[i])
                ok = 0;
        }
        if (ok)
            out = eval(X, D->body, argv);
        for (int i = 0; i < e->nargs; i++)
            free(argv[i]);
        return out;
    }
    }
    X->rc = ORC_EINVAL;
    return NULL;
}

/* Number of outputs in src (parse only), or a negative error code. */
int oracle_count_outputs(const char *src, char *err, int errlen)
{
    Prog G;
    memset(&G, 0, sizeof G);
    int rc = parse_program(src, &G, err, errlen);
    int nout = G.noutputs;
    free_prog(&G);
    return rc == ORC_OK ? nout : rc;
}

/* Evaluate every output of src on img ([C][D][H][W]).  Output i is written
 * to out + i*D*H*W (one byte per voxel) for i < max_out.  Returns the number
 * of outputs, or a negative error code (message in err). */
int oracle_run3(const char *src, const void *img, int dtype, int C, int D, int H, int W, uint8_t *out,
                int max_out, char *err, int errlen)
{
    if (err && errlen > 0)
        err[0] = 0;
    if ((dtype != DT_F32 && dtype != DT_U8 && dtype != DT_U16) || C < 1 || D < 1 || H < 0 || W < 0) {
        if (err && errlen > 0)
            snprintf(err, (size_t)errlen, "bad image description");
        return ORC_EINVAL;
    }
    Prog G;
    memset(&G, 0, sizeof G);
    int rc = parse_program(src, &G, err, errlen);
    if (rc != ORC_OK) {
        free_prog(&G);
        return rc;
    }
    Ctx X;
    memset(&X, 0, sizeof X);
    X.G = &G;
    X.img = img;
    X.dtype = dtype;
    X.C = C;
    X.D = D;
    X.H = H;
    X.W = W;
    X.n = (int64_t)D * H * W;
    X.err = err;
    X.errlen = errlen;
    X.rc = ORC_OK;
    int oi = 0;
    for (int s = 0; s < G.nstmts && X.rc == ORC_OK; s++) {
        Stmt *S = &G.stmts[s];
        if (!S->is_output) {
            Def *D = &G.defs[S->def];
            if (D->nparams > 0)
                continue;                 /* macros are expanded at each call */
            if (D->refs_left == 0 && !D->pinned) {
                D->evaluated = 1;         /* never read: skip */
                continue;
            }
            D->value = eval(&X, D->body, NULL);
            D->evaluated = 1;
        } else {
            uint8_t *m = eval(&X, S->expr, NULL);
            if (m && oi < max_out && out)
                memcpy(out + (int64_t)oi * X.n, m, (size_t)X.n);
            free(m);
            oi++;
        }
    }
    rc = X.rc;
    free_prog(&G);
    return rc == ORC_OK ? oi : rc;
}

/* A 2-D image: one slice. */
int oracle_run(const char *src, const void *img, int dtype, int C, int H, int W, uint8_t *out,
               int max_out, char *err, int errlen)
{
    return oracle_run3(src, img, dtype, C, 1, H, W, out, max_out, err, errlen);
}
