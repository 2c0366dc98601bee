/* Host AddressSanitizer / UndefinedBehaviorSanitizer run of the CPU oracle:
 * every entry point on small and ragged sizes (1 x 1 up to non-square,
 * non-power-of-two images), so out-of-bounds indexing, signed overflow or
 * uninitialised reads in the oracle show up as sanitizer reports.  Built and
 * run by tests/test_sanitizers.py; exits non-zero on a bad status. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int64_t oracle_next_pow2(int64_t v);
int oracle_quadrant(const double* img, int64_t w, int64_t h, int64_t ld, int q, int single, double* out);
int oracle_quadrant_op(const double* img, int64_t w, int64_t h, int64_t ld, int q, int op, double* out);
int oracle_full(const double* img, int64_t w, int64_t h, int64_t ld, int single, double* out);
int oracle_full_op(const double* img, int64_t w, int64_t h, int64_t ld, int op, double* out);
int oracle_fhtshift_full(const double* in, int64_t w, int64_t h, int inverse, double* out);
int oracle_range(const double* img, int64_t w, int64_t h, int64_t ld, int64_t S1, int64_t S, int transposed,
                 int single, double* out);
int oracle_range_scaled(const double* img, int64_t w, int64_t h, int64_t ld, int64_t num, int64_t den, int64_t S1,
                        int64_t S, int transposed, int single, double* out);
double oracle_cell(const double* img, int64_t w, int64_t h, int64_t ld, int q, int64_t s, int64_t x);
double oracle_full_cell(const double* img, int64_t w, int64_t h, int64_t ld, int64_t r, int64_t x);
int oracle_adjoint_full(const double* g, int64_t w, int64_t h, int single, double* out, int64_t ld_out);
int oracle_adjoint_quadrant(const double* g, int64_t w, int64_t h, int q, int single, double* out, int64_t ld_out);
int oracle_range_adjoint(const double* g, int64_t w, int64_t h, int64_t S1, int64_t S, int transposed, int single,
                         double* out, int64_t ld_out);

static int fails = 0;
#define CHECK(x) do { if ((x) != 0) { printf("bad status at %s:%d\n", __FILE__, __LINE__); ++fails; } } while (0)

int main(void)
{
    const int64_t sizes[][2] = {{1, 1}, {1, 2}, {2, 1}, {3, 5}, {5, 3}, {7, 12}, {16, 9}, {13, 32}, {33, 17}};
    for (size_t i = 0; i < sizeof sizes / sizeof sizes[0]; ++i) {
        const int64_t h = sizes[i][0], w = sizes[i][1];
        const int64_t hp = oracle_next_pow2(h), wp = oracle_next_pow2(w), W = hp + wp;
        const int64_t rows = 2 * (hp + wp) - 3, nmax = hp > wp ? hp : wp;
        double* img = malloc(sizeof(double) * (size_t)(h * w));
        double* q = malloc(sizeof(double) * (size_t)(nmax * W));
        double* f = malloc(sizeof(double) * (size_t)(rows * W));
        double* f2 = malloc(sizeof(double) * (size_t)(rows * W));
        double* g = malloc(sizeof(double) * (size_t)(h * w));
        for (int64_t k = 0; k < h * w; ++k) img[k] = (double)((k * 7 + 3) % 11);
        for (int qq = 1; qq <= 4; ++qq) {
            CHECK(oracle_quadrant(img, w, h, w, qq, 0, q));
            CHECK(oracle_quadrant(img, w, h, w, qq, 1, q));
            CHECK(oracle_quadrant_op(img, w, h, w, qq, 1, q));
            CHECK(oracle_adjoint_quadrant(q, w, h, qq, 1, g, w));
            for (int64_t s = 0; s < (qq <= 2 ? hp : wp); ++s)
                for (int64_t x = 0; x < W; x += 3) (void)oracle_cell(img, w, h, w, qq, s, x);
        }
        CHECK(oracle_full(img, w, h, w, 0, f));
        CHECK(oracle_full(img, w, h, w, 1, f));
        CHECK(oracle_full_op(img, w, h, w, 1, f));
        CHECK(oracle_fhtshift_full(f, w, h, 0, f2));
        CHECK(oracle_fhtshift_full(f2, w, h, 1, f));
        for (int64_t r = 0; r < rows; ++r) (void)oracle_full_cell(img, w, h, w, r, (r * 5) % W);
        if (!isnan(oracle_full_cell(img, w, h, w, rows, 0))) { printf("row past the image\n"); ++fails; }
        CHECK(oracle_adjoint_full(f, w, h, 0, g, w));
        CHECK(oracle_adjoint_full(f, w, h, 1, g, w));
        for (int tr = 0; tr < 2; ++tr) {
            const int64_t n = tr ? wp : hp;
            const int64_t S1s[] = {0, n - 1, -(n - 1), (n - 1) / 2};
            for (int k = 0; k < 4; ++k) {
                const int64_t S = n - 1;
                CHECK(oracle_range(img, w, h, w, S1s[k], S, tr, 0, q));
                CHECK(oracle_range_adjoint(q, w, h, S1s[k], S, tr, 1, g, w));
            }
            /* scaled by 3/2 and 1/2 along the sheared axis */
            const int64_t ws = tr ? w : (w * 3 + 1) / 2, hs = tr ? (h * 3 + 1) / 2 : h;
            const int64_t Wsc = oracle_next_pow2(ws) + oracle_next_pow2(hs);
            const int64_t ns = tr ? oracle_next_pow2(ws) : oracle_next_pow2(hs);
            double* rs = malloc(sizeof(double) * (size_t)(ns * Wsc));
            CHECK(oracle_range_scaled(img, w, h, w, 3, 2, 0, ns - 1, tr, 0, rs));
            free(rs);
        }
        /* invalid arguments are rejected, not dereferenced */
        if (oracle_quadrant(img, w, h, w - 1, 1, 0, q) == 0 && w > 1) { printf("ld < w accepted\n"); ++fails; }
        if (oracle_range(img, w, h, w, hp, 0, 0, 0, q) == 0 && hp > 1) { printf("|S1| > n-1 accepted\n"); ++fails; }
        free(img); free(q); free(f); free(f2); free(g);
    }
    printf("oracle sanitizer run: %s\n", fails ? "FAILED" : "clean");
    return fails ? 1 : 0;
}
