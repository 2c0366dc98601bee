/*
 * CPU oracle for the Brady dyadic Fast Hough Transform, as studied in
 * Aliev, Ershov, Nikolaev, "On the use of FHT, its modification for practical
 * applications and the structure of Hough image" (arXiv 1811.06378).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the HIP
 * path.
 *
 * Plain and slow on purpose: every routine follows the definition or the
 * algorithm step by step, in double precision.  The optional single-precision
 * mode rounds every addition of the stage recurrence to binary32, which gives
 * exactly the binary32 sum of the same two operands (double rounding is
 * innocuous for addition when 53 >= 2*24+2, Figueroa 1995), i.e. the same add
 * tree evaluated in float.
 *
 * Conventions (the paper leaves them implicit; the readings are listed with the
 * design notes):
 *   image I: h rows x w columns, I[y*ld + x];  h' = 2^ceil(log2 h),
 *   w' = 2^ceil(log2 w), W = w' + h'.
 *   P  (h' x W): I zero-padded on the right and bottom (section 3.1: the
 *                extension by an h x h zero block that keeps patterns from
 *                flowing through the boundary; pow2 padding of both sides).
 *   Pt (w' x W): the transposed image padded the same way (section 3.1: mostly
 *                horizontal lines are handled on the transposed image).
 *   D_n(s, y):   column offset at row y of the dyadic pattern with shift s
 *                over n = 2^k rows (Brady's pattern, section 2).
 *   quadrant 1:  H1[s,x] = sum_y P [y, (x + D_h'(s,y)) mod W]
 *   quadrant 2:  H2[s,x] = sum_y P [y, (x - D_h'(s,y)) mod W]
 *   quadrant 3:  H3[s,x] = sum_c Pt[c, (x - D_w'(s,c)) mod W]
 *   quadrant 4:  H4[s,x] = sum_c Pt[c, (x + D_w'(s,c)) mod W]
 *   full image:  [flip(H1); H2[1:]; flip(H3)[1:]; H4[1:]], 2(w'+h')-3 rows
 *                (section 3.3).
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_BAD_ARG -1
#define ORACLE_NO_MEMORY -2

/* operation along the patterns: the sum of the paper, or max (section 1
   notes the transform generalises to any associative, commutative op) */
#define ORACLE_OP_SUM 0
#define ORACLE_OP_MAX 1

/* Threads the OpenMP loops use (1 without OpenMP). */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int64_t oracle_next_pow2(int64_t v)
{
    int64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

static int64_t mod_w(int64_t a, int64_t W)
{
    int64_t r = a % W;
    return r < 0 ? r + W : r;
}

/* floor(a / b) for b > 0 (C division truncates toward zero). */
static int64_t floor_div(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b != 0) && (a < 0)) q -= 1;
    return q;
}

/*
 * D_n(s, y), section 2 (Brady's dyadic pattern) and the block iteration of
 * section 4 (Fig. 6): a pattern of n rows with shift s is the top half with
 * shift s>>1 followed by the bottom half with shift s>>1 that starts
 * s - (s>>1) columns further right.  Written as the recursion it is.
 */
int64_t oracle_pattern_offset(int64_t n, int64_t s, int64_t y)
{
    if (n <= 1) return 0;
    int64_t half = n / 2;
    int64_t sub = s >> 1;
    if (y < half) return oracle_pattern_offset(half, sub, y);
    return (s - sub) + oracle_pattern_offset(half, sub, y - half);
}

/* Quadrant geometry: source is P (q = 1, 2) or Pt (q = 3, 4); direction is
 * +1 for q = 1, 4 and -1 for q = 2, 3 (section 3.1 quadrant list). */
static int quadrant_dir(int q) { return (q == 1 || q == 4) ? 1 : -1; }
static int quadrant_transposed(int q) { return q >= 3; }

/* Value of the padded source array (P or Pt) at (r, c), 0 outside I. */
static double src_value(const double* img, int64_t w, int64_t h, int64_t ld, int transposed,
                        int64_t r, int64_t c)
{
    int64_t y = transposed ? c : r;
    int64_t x = transposed ? r : c;
    if (y < 0 || y >= h || x < 0 || x >= w) return 0.0;
    return img[y * ld + x];
}

/*
 * Stage recurrence of one quadrant (section 2 and section 4, Fig. 6): after
 * stage j the rows are grouped in blocks of 2^(j+1); row t of a block holds the
 * sums along all patterns with shift t over the block's rows.  Stage j merges
 * two adjacent blocks of 2^j rows:
 *   A[j+1][b*2^(j+1) + t][x] = A[j][b*2^(j+1) + (t>>1)][x]
 *                            + A[j][b*2^(j+1) + 2^j + (t>>1)][x + dir*(t - (t>>1))]
 * (column index mod W).  `pre_shift` (may be NULL) rolls source row r right
 * by pre_shift[r] columns before the first stage (section 4: the rows of the
 * first iteration are read as if already cyclically shifted).
 * out: n x W, row-major, n = h' (q=1,2) or w' (q=3,4).
 */
static int quadrant_recurrence(const double* img, int64_t w, int64_t h, int64_t ld, int q,
                               int single, int op, const int64_t* pre_shift, double* out)
{
    int64_t hp = oracle_next_pow2(h), wp = oracle_next_pow2(w);
    int64_t W = hp + wp;
    int transposed = quadrant_transposed(q);
    int dir = quadrant_dir(q);
    int64_t n = transposed ? wp : hp;

    double* a = (double*)malloc(sizeof(double) * (size_t)(n * W));
    double* b = (double*)malloc(sizeof(double) * (size_t)(n * W));
    if (!a || !b) { free(a); free(b); return ORACLE_NO_MEMORY; }

    for (int64_t r = 0; r < n; ++r) {
        int64_t roll = pre_shift ? pre_shift[r] : 0;
        for (int64_t x = 0; x < W; ++x)
            a[r * W + x] = src_value(img, w, h, ld, transposed, r, mod_w(x - roll, W));
    }

    for (int64_t blk = 1; blk < n; blk *= 2) {            /* blk = 2^j */
        int64_t pair = 2 * blk;
        #pragma omp parallel for schedule(static)
        for (int64_t row = 0; row < n; ++row) {
            int64_t base = (row / pair) * pair;
            int64_t t = row - base;
            int64_t sub = t >> 1;
            const double* top = a + (base + sub) * W;
            const double* bot = a + (base + blk + sub) * W;
            int64_t off = dir * (t - sub);
            double* dst = b + row * W;
            for (int64_t x = 0; x < W; ++x) {
                double v;
                if (op == ORACLE_OP_MAX) {
                    /* section 1: the same patterns under another associative,
                       commutative operation; max is exact in any precision */
                    double u = bot[mod_w(x + off, W)];
                    v = top[x] > u ? top[x] : u;
                } else {
                    v = top[x] + bot[mod_w(x + off, W)];
                    if (single) v = (double)(float)v;
                }
                dst[x] = v;
            }
        }
        double* tmp = a; a = b; b = tmp;
    }
    memcpy(out, a, sizeof(double) * (size_t)(n * W));
    free(a);
    free(b);
    return ORACLE_OK;
}

static int quadrant_op(const double* img, int64_t w, int64_t h, int64_t ld, int q, int single, int op,
                       double* out)
{
    if (!img || !out || w < 1 || h < 1 || ld < w || q < 1 || q > 4) return ORACLE_BAD_ARG;
    if (op != ORACLE_OP_SUM && op != ORACLE_OP_MAX) return ORACLE_BAD_ARG;
    if (single) {
        /* single-precision mode takes binary32 inputs */
        for (int64_t y = 0; y < h; ++y)
            for (int64_t x = 0; x < w; ++x)
                if ((double)(float)img[y * ld + x] != img[y * ld + x]) return ORACLE_BAD_ARG;
    }
    return quadrant_recurrence(img, w, h, ld, q, single, op, NULL, out);
}

/* One quadrant, q in 1..4, out n x W (n = h' for q = 1, 2; w' for q = 3, 4). */
int oracle_quadrant(const double* img, int64_t w, int64_t h, int64_t ld, int q, int single,
                    double* out)
{
    return quadrant_op(img, w, h, ld, q, single, ORACLE_OP_SUM, out);
}

/* The same quadrant with op = ORACLE_OP_SUM (0) or ORACLE_OP_MAX (1). */
int oracle_quadrant_op(const double* img, int64_t w, int64_t h, int64_t ld, int q, int op, double* out)
{
    return quadrant_op(img, w, h, ld, q, 0, op, out);
}

/*
 * Full Hough image, section 3.3: quadrant 1 flipped vertically, quadrant 2,
 * quadrant 3 flipped, quadrant 4, each join sharing one row (the shared rows
 * are equal, so the second copy is dropped).  out: (2(w'+h')-3) x W.
 */
static int full_op(const double* img, int64_t w, int64_t h, int64_t ld, int single, int op, double* out)
{
    if (!img || !out || w < 1 || h < 1 || ld < w) return ORACLE_BAD_ARG;
    int64_t hp = oracle_next_pow2(h), wp = oracle_next_pow2(w);
    int64_t W = hp + wp;
    double* hq = (double*)malloc(sizeof(double) * (size_t)((hp > wp ? hp : wp) * W));
    if (!hq) return ORACLE_NO_MEMORY;
    int64_t row = 0;
    for (int q = 1; q <= 4; ++q) {
        int rc = quadrant_op(img, w, h, ld, q, single, op, hq);
        if (rc) { free(hq); return rc; }
        int64_t n = (q <= 2) ? hp : wp;
        int flip = (q == 1 || q == 3);
        int64_t first = (q == 1) ? 0 : 1;      /* drop the row shared with the previous quadrant */
        for (int64_t i = first; i < n; ++i) {
            int64_t s = flip ? (n - 1 - i) : i;
            memcpy(out + row * W, hq + s * W, sizeof(double) * (size_t)W);
            ++row;
        }
    }
    free(hq);
    return ORACLE_OK;
}

int oracle_full(const double* img, int64_t w, int64_t h, int64_t ld, int single, double* out)
{
    return full_op(img, w, h, ld, single, ORACLE_OP_SUM, out);
}

/* Full image of the max transform (section 1): same layout, max for sum. */
int oracle_full_op(const double* img, int64_t w, int64_t h, int64_t ld, int op, double* out)
{
    return full_op(img, w, h, ld, 0, op, out);
}

/*
 * Quadrant and local shift of a full-image row (section 3.3, closing
 * paragraph): rows [0, h') are quadrant 1 (flipped), [h', 2h'-1) quadrant 2,
 * [2h'-1, 2h'+w'-2) quadrant 3 (flipped), the rest quadrant 4.
 */
int oracle_row_quadrant(int64_t w, int64_t h, int64_t r, int64_t* s_out)
{
    int64_t hp = oracle_next_pow2(h), wp = oracle_next_pow2(w);
    int64_t rows = 2 * (hp + wp) - 3;
    if (r < 0 || r >= rows) return 0;
    if (r < hp) { *s_out = hp - 1 - r; return 1; }
    if (r < 2 * hp - 1) { *s_out = r - hp + 1; return 2; }
    if (r < 2 * hp + wp - 2) { *s_out = 2 * hp + wp - 3 - r; return 3; }
    *s_out = r - (2 * hp + wp - 3);
    return 4;
}

/*
 * fhtshift, section 5: every row is rolled cyclically (towards larger x0) so
 * that its meaningful run of w'+s (vertical) or h'+s (horizontal) cells is
 * centred in the W columns; the black zone then sits at both edges.  The
 * meaningful run of quadrant 1 row s starts at x0 = -s, of quadrant 2 at 0,
 * of quadrant 3 at 0, of quadrant 4 at -s; centring it gives the roll amounts
 *   q1: floor((h'+s)/2), q2: floor((h'-s)/2), q3: floor((w'-s)/2),
 *   q4: floor((w'+s)/2).
 * (The paper's continuous h - i/2 for the flipped quadrant 1 is the q1 case.)
 */
int64_t oracle_fhtshift_roll(int q, int64_t hp, int64_t wp, int64_t s)
{
    switch (q) {
    case 1: return (hp + s) / 2;
    case 2: return (hp - s) / 2;
    case 3: return (wp - s) / 2;
    case 4: return (wp + s) / 2;
    default: return 0;
    }
}

/* Apply (inverse = 0) or undo (inverse = 1) fhtshift on a full Hough image. */
int oracle_fhtshift_full(const double* in, int64_t w, int64_t h, int inverse, double* out)
{
    if (!in || !out || w < 1 || h < 1) return ORACLE_BAD_ARG;
    int64_t hp = oracle_next_pow2(h), wp = oracle_next_pow2(w);
    int64_t W = hp + wp, rows = 2 * (hp + wp) - 3;
    for (int64_t r = 0; r < rows; ++r) {
        int64_t s = 0;
        int q = oracle_row_quadrant(w, h, r, &s);
        int64_t roll = oracle_fhtshift_roll(q, hp, wp, s);
        if (inverse) roll = -roll;
        for (int64_t x = 0; x < W; ++x)
            out[r * W + mod_w(x + roll, W)] = in[r * W + x];
    }
    return ORACLE_OK;
}

/*
 * Angle-range variant, section 4.  A horizontal shear maps an inclination range
 * onto one quadrant; the shear is applied by reading the rows of the first
 * iteration cyclically pre-shifted.  Integer form: the range is shifts
 * s = 0..S of a pattern whose slope is (s - S1)/(n-1) columns per row, so row
 * y of the source is rolled right (towards larger x) by sigma(y) with
 *   sigma(y) = floor((2*y*S1 + (n-1)) / (2*(n-1)))   (y*S1/(n-1) rounded half up),
 * and the result is rows 0..S of quadrant 1 (quadrant 4 when transposed) of
 * the sheared image.  Requires 0 <= S <= n-1, |S1| <= n-1.
 * out: (S+1) x W.
 */
int64_t oracle_range_sigma(int64_t n, int64_t S1, int64_t y)
{
    if (n <= 1) return 0;
    return floor_div(2 * y * S1 + (n - 1), 2 * (n - 1));
}

int oracle_range(const double* img, int64_t w, int64_t h, int64_t ld, int64_t S1, int64_t S,
                 int transposed, int single, double* out)
{
    if (!img || !out || w < 1 || h < 1 || ld < w) return ORACLE_BAD_ARG;
    int64_t hp = oracle_next_pow2(h), wp = oracle_next_pow2(w);
    int64_t W = hp + wp;
    int64_t n = transposed ? wp : hp;
    if (S < 0 || S > n - 1 || S1 > n - 1 || S1 < -(n - 1)) return ORACLE_BAD_ARG;
    int64_t* roll = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    double* hq = (double*)malloc(sizeof(double) * (size_t)(n * W));
    if (!roll || !hq) { free(roll); free(hq); return ORACLE_NO_MEMORY; }
    for (int64_t y = 0; y < n; ++y) roll[y] = oracle_range_sigma(n, S1, y);
    int rc = quadrant_recurrence(img, w, h, ld, transposed ? 4 : 1, single, ORACLE_OP_SUM, roll, hq);
    if (rc == ORACLE_OK) memcpy(out, hq, sizeof(double) * (size_t)((S + 1) * W));
    free(roll);
    free(hq);
    return rc;
}

/*
 * Angle range of the image scaled along the axis the range shears (image
 * columns; image rows when transposed) by alpha = num/den (section 4: a
 * scale maps [-arctg(1/alpha); 0] onto [-45; 0], done in the first
 * iteration).  The paper fixes no resampling rule; this reading takes the
 * nearest source sample: the scaled image has ceil(alpha * extent) samples
 * along that axis and sample x is source sample floor(x * den / num).  The
 * scaled image is built explicitly, then transformed by oracle_range.
 * out: (S+1) x W_alpha with W_alpha from the scaled sizes.
 */
int oracle_range_scaled(const double* img, int64_t w, int64_t h, int64_t ld, int64_t num, int64_t den,
                        int64_t S1, int64_t S, int transposed, int single, double* out)
{
    if (!img || !out || w < 1 || h < 1 || ld < w || num < 1 || den < 1) return ORACLE_BAD_ARG;
    int64_t ws = transposed ? w : (w * num + den - 1) / den;
    int64_t hs = transposed ? (h * num + den - 1) / den : h;
    double* sc = (double*)malloc(sizeof(double) * (size_t)(ws * hs));
    if (!sc) return ORACLE_NO_MEMORY;
    for (int64_t y = 0; y < hs; ++y)
        for (int64_t x = 0; x < ws; ++x) {
            int64_t sy = transposed ? (y * den) / num : y;
            int64_t sx = transposed ? x : (x * den) / num;
            sc[y * ws + x] = img[sy * ld + sx];
        }
    int rc = oracle_range(sc, ws, hs, ws, S1, S, transposed, single, out);
    free(sc);
    return rc;
}

/*
 * One Hough cell by its definition: the sum of the padded source along one
 * dyadic pattern, H_q[s, x] = sum_r src[r, (x + dir*D_n(s, r)) mod W].
 * Used for sampled checks at sizes where the full oracle is too slow.
 */
double oracle_cell(const double* img, int64_t w, int64_t h, int64_t ld, int q, int64_t s,
                   int64_t x)
{
    int64_t hp = oracle_next_pow2(h), wp = oracle_next_pow2(w);
    int64_t W = hp + wp;
    int transposed = quadrant_transposed(q);
    int dir = quadrant_dir(q);
    int64_t n = transposed ? wp : hp;
    double acc = 0.0;
    for (int64_t r = 0; r < n; ++r)
        acc += src_value(img, w, h, ld, transposed, r,
                         mod_w(x + dir * oracle_pattern_offset(n, s, r), W));
    return acc;
}

/* Same for a full-image cell (row r of the assembled image). */
double oracle_full_cell(const double* img, int64_t w, int64_t h, int64_t ld, int64_t r, int64_t x)
{
    int64_t s = 0;
    int q = oracle_row_quadrant(w, h, r, &s);
    if (q == 0) return NAN;
    return oracle_cell(img, w, h, ld, q, s, x);
}

/*
 * Adjoint (transpose) of one quadrant: given a gradient g on the n x W
 * quadrant, returns the gradient on the padded source, by running the stage
 * recurrence backwards.  The transpose of one stage sends each output row t of
 * a merged block back to the two rows it was summed from:
 *   top row t>>1    gets g[t][x]
 *   bottom row t>>1 gets g[t][x - dir*(t - (t>>1))]
 * so, collecting by input row u of each half,
 *   top[u][x]    = g[2u][x] + g[2u+1][x]
 *   bottom[u][x] = g[2u][x - dir*u] + g[2u+1][x - dir*(u+1)].
 * out: n x W on the padded source.
 */
static int quadrant_adjoint(const double* g, int64_t n, int64_t W, int dir, int single, double* out)
{
    double* a = (double*)malloc(sizeof(double) * (size_t)(n * W));
    double* b = (double*)malloc(sizeof(double) * (size_t)(n * W));
    if (!a || !b) { free(a); free(b); return ORACLE_NO_MEMORY; }
    memcpy(a, g, sizeof(double) * (size_t)(n * W));
    for (int64_t blk = n / 2; blk >= 1; blk /= 2) {       /* undo the stage that merged blocks of blk */
        int64_t pair = 2 * blk;
        #pragma omp parallel for schedule(static)
        for (int64_t row = 0; row < n; ++row) {
            int64_t base = (row / pair) * pair;
            int64_t i = row - base;
            double* dst = b + row * W;
            if (i < blk) {
                const double* g0 = a + (base + 2 * i) * W;
                const double* g1 = a + (base + 2 * i + 1) * W;
                for (int64_t x = 0; x < W; ++x) {
                    double v = g0[x] + g1[x];
                    if (single) v = (double)(float)v;
                    dst[x] = v;
                }
            } else {
                int64_t u = i - blk;
                const double* g0 = a + (base + 2 * u) * W;
                const double* g1 = a + (base + 2 * u + 1) * W;
                for (int64_t x = 0; x < W; ++x) {
                    double v = g0[mod_w(x - dir * u, W)] + g1[mod_w(x - dir * (u + 1), W)];
                    if (single) v = (double)(float)v;
                    dst[x] = v;
                }
            }
        }
        double* tmp = a; a = b; b = tmp;
    }
    memcpy(out, a, sizeof(double) * (size_t)(n * W));
    free(a);
    free(b);
    return ORACLE_OK;
}

/*
 * Adjoint of the full Hough image: the gradient of every full-image row goes
 * to the one quadrant row it was copied from (the dropped duplicate rows get
 * nothing), each quadrant is transposed back to its padded source, and the
 * four contributions are summed on the h x w image (padding cropped).
 * g: (2(w'+h')-3) x W;  out: h x w, row-major with ld_out.
 */
int oracle_adjoint_full(const double* g, int64_t w, int64_t h, int single, double* out,
                        int64_t ld_out)
{
    if (!g || !out || w < 1 || h < 1 || ld_out < w) return ORACLE_BAD_ARG;
    int64_t hp = oracle_next_pow2(h), wp = oracle_next_pow2(w);
    int64_t W = hp + wp, rows = 2 * (hp + wp) - 3;
    int64_t nmax = hp > wp ? hp : wp;
    double* slab = (double*)malloc(sizeof(double) * (size_t)(nmax * W));
    double* src = (double*)malloc(sizeof(double) * (size_t)(nmax * W));
    if (!slab || !src) { free(slab); free(src); return ORACLE_NO_MEMORY; }
    for (int64_t y = 0; y < h; ++y)
        for (int64_t x = 0; x < w; ++x) out[y * ld_out + x] = 0.0;
    for (int q = 1; q <= 4; ++q) {
        int64_t n = (q <= 2) ? hp : wp;
        memset(slab, 0, sizeof(double) * (size_t)(n * W));
        for (int64_t r = 0; r < rows; ++r) {
            int64_t s = 0;
            if (oracle_row_quadrant(w, h, r, &s) == q)
                memcpy(slab + s * W, g + r * W, sizeof(double) * (size_t)W);
        }
        int rc = quadrant_adjoint(slab, n, W, quadrant_dir(q), single, src);
        if (rc) { free(slab); free(src); return rc; }
        for (int64_t y = 0; y < h; ++y)
            for (int64_t x = 0; x < w; ++x) {
                double v = quadrant_transposed(q) ? src[x * W + y] : src[y * W + x];
                double acc = out[y * ld_out + x] + v;
                if (single) acc = (double)(float)acc;
                out[y * ld_out + x] = acc;
            }
    }
    free(slab);
    free(src);
    return ORACLE_OK;
}

/*
 * Adjoint of the angle-range transform (section 4).  The range output is rows
 * 0..S of quadrant 1 (4 when transposed) of the padded source whose row r is
 * rolled right by sigma(r); so the gradient rows 0..S (rows S+1..n-1 get
 * none) go back through the transposed stages to that sheared source, whose
 * cell (r, xi) is the source cell (r, xi - sigma(r)); the result is cropped
 * to the h x w image (transposed back for the mostly-horizontal variant).
 * g: (S+1) x W;  out: h x w, row-major with ld_out.
 */
int oracle_range_adjoint(const double* g, int64_t w, int64_t h, int64_t S1, int64_t S, int transposed,
                         int single, double* out, int64_t ld_out)
{
    if (!g || !out || w < 1 || h < 1 || ld_out < w) return ORACLE_BAD_ARG;
    int64_t hp = oracle_next_pow2(h), wp = oracle_next_pow2(w);
    int64_t W = hp + wp;
    int64_t n = transposed ? wp : hp;
    if (S < 0 || S > n - 1 || S1 > n - 1 || S1 < -(n - 1)) return ORACLE_BAD_ARG;
    double* slab = (double*)calloc((size_t)(n * W), sizeof(double));
    double* src = (double*)malloc(sizeof(double) * (size_t)(n * W));
    if (!slab || !src) { free(slab); free(src); return ORACLE_NO_MEMORY; }
    memcpy(slab, g, sizeof(double) * (size_t)((S + 1) * W));
    int rc = quadrant_adjoint(slab, n, W, +1, single, src);
    if (rc == ORACLE_OK)
        for (int64_t y = 0; y < h; ++y)
            for (int64_t x = 0; x < w; ++x) {
                int64_t r = transposed ? x : y;     /* source row (image row, or column) */
                int64_t c = transposed ? y : x;     /* source column */
                out[y * ld_out + x] = src[r * W + mod_w(c + oracle_range_sigma(n, S1, r), W)];
            }
    free(slab);
    free(src);
    return rc;
}

/* Adjoint of one quadrant alone (gradient n x W) onto the h x w image. */
int oracle_adjoint_quadrant(const double* g, int64_t w, int64_t h, int q, int single, double* out,
                            int64_t ld_out)
{
    if (!g || !out || w < 1 || h < 1 || ld_out < w || q < 1 || q > 4) return ORACLE_BAD_ARG;
    int64_t hp = oracle_next_pow2(h), wp = oracle_next_pow2(w);
    int64_t W = hp + wp;
    int64_t n = (q <= 2) ? hp : wp;
    double* src = (double*)malloc(sizeof(double) * (size_t)(n * W));
    if (!src) return ORACLE_NO_MEMORY;
    int rc = quadrant_adjoint(g, n, W, quadrant_dir(q), single, src);
    if (rc == ORACLE_OK)
        for (int64_t y = 0; y < h; ++y)
            for (int64_t x = 0; x < w; ++x)
                out[y * ld_out + x] = quadrant_transposed(q) ? src[x * W + y] : src[y * W + x];
    free(src);
    return rc;
}
