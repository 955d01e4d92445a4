/*
 * quant.c -- reference encoders/decoders for the low-precision operand
 * formats of the mixed-precision trailing update, and the per-tile
 * power-of-two scale rule.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.c).  Written from the format
 * definitions, with the rounding done by exact arithmetic on binary64
 * values (rint() in the default round-to-nearest-even mode):
 *
 *   BF16   : 1 sign, 8 exponent (bias 127), 7 fraction bits; the upper half
 *            of an IEEE binary32.  Encoded from a binary32 value.
 *   FP16   : IEEE binary16, 1/5/10, bias 15, subnormals, max 65504.
 *   E4M3FN : OCP 8-bit float, 1/4/3, bias 7, subnormals, no infinities,
 *            S.1111.111 is NaN, max finite 448.  Encoding saturates to
 *            +-448 (values beyond the range never occur after scaling).
 *
 * Tile scale: for a tile with largest magnitude amax > 0, the scale is 2^e
 * with e = floor(log2(maxfinite / amax)), computed exactly from the binary32
 * exponent and fraction of amax (no division), capped at 64; amax == 0
 * gives e = 0.  Scaled values amax * 2^e then lie in (maxfinite/2,
 * maxfinite].  BF16 keeps binary32's exponent range and uses no scale.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#include <stddef.h>

enum { FMT_BF16 = 1, FMT_FP16 = 2, FMT_E4M3 = 3 };

static uint32_t f32_bits(float x) { uint32_t u; memcpy(&u, &x, 4); return u; }

uint16_t oracle_enc_bf16(float x)
{
    uint32_t u = f32_bits(x);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu))
        return (uint16_t)((u >> 16) | 0x0040u);            /* quiet NaN */
    /* Round the low 16 bits to nearest, ties to even, by exact arithmetic. */
    uint32_t hi = u >> 16, lo = u & 0xffffu;
    if (lo > 0x8000u || (lo == 0x8000u && (hi & 1u))) hi += 1u;
    return (uint16_t)hi;
}

double oracle_dec_bf16(uint16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float f; memcpy(&f, &u, 4);
    return (double)f;
}

/* Round |v| to a multiple of the quantum 2^qexp, ties to even. */
static double round_to_quantum(double a, int qexp)
{
    return ldexp(rint(ldexp(a, -qexp)), qexp);
}

uint16_t oracle_enc_f16(double v)
{
    uint16_t s = signbit(v) ? 0x8000u : 0u;
    double a = fabs(v);
    if (isnan(v)) return 0x7e00u;
    /* quantum: 2^(e-10) for normals (e >= -14), 2^-24 for subnormals */
    int e = a > 0 ? ilogb(a) : -25;
    int qexp = (e >= -14 ? e : -14) - 10;
    double r = round_to_quantum(a, qexp);
    if (r > 65504.0) return s | 0x7c00u;                   /* overflow: inf */
    if (r == 0.0) return s;
    int er = ilogb(r);
    if (er < -14)                                          /* subnormal */
        return s | (uint16_t)ldexp(r, 24);
    uint16_t frac = (uint16_t)(ldexp(r, -er) * 1024.0 - 1024.0);
    return s | (uint16_t)((er + 15) << 10) | frac;
}

double oracle_dec_f16(uint16_t h)
{
    int s = h >> 15, e = (h >> 10) & 0x1f, f = h & 0x3ff;
    double v;
    if (e == 0) v = ldexp((double)f, -24);
    else if (e == 31) v = f ? NAN : INFINITY;
    else v = ldexp(1.0 + f / 1024.0, e - 15);
    return s ? -v : v;
}

uint8_t oracle_enc_e4m3(double v)
{
    uint8_t s = signbit(v) ? 0x80u : 0u;
    double a = fabs(v);
    if (isnan(v)) return 0x7fu;
    if (a >= 448.0) return s | 0x7eu;                      /* saturate */
    int e = a > 0 ? ilogb(a) : -10;
    int qexp = (e >= -6 ? e : -6) - 3;
    double r = round_to_quantum(a, qexp);
    if (r > 448.0) r = 448.0;
    if (r == 0.0) return s;
    int er = ilogb(r);
    if (er < -6)                                           /* subnormal */
        return s | (uint8_t)ldexp(r, 9);
    uint8_t frac = (uint8_t)(ldexp(r, -er) * 8.0 - 8.0);
    return s | (uint8_t)((er + 7) << 3) | frac;
}

double oracle_dec_e4m3(uint8_t c)
{
    int s = c >> 7, e = (c >> 3) & 0xf, f = c & 7;
    double v;
    if (e == 15 && f == 7) v = NAN;
    else if (e == 0) v = ldexp((double)f, -9);
    else v = ldexp(1.0 + f / 8.0, e - 7);
    return s ? -v : v;
}

/* Scale exponent e for a tile of largest magnitude amax (see header). */
int oracle_tile_scale_exp(int fmt, float amax)
{
    if (fmt == FMT_BF16) return 0;
    if (!(amax > 0.0f)) return 0;
    /* maxfinite = mf * 2^Ef with mf in [1,2); amax = ma * 2^Ea likewise. */
    int Ef = fmt == FMT_FP16 ? 15 : 8;
    double mf = fmt == FMT_FP16 ? 65504.0 / 32768.0 : 448.0 / 256.0;
    int Ea = ilogb((double)amax);
    double ma = ldexp((double)amax, -Ea);
    int e = Ef - Ea - (ma > mf ? 1 : 0);
    return e > 64 ? 64 : e;
}

/*
 * Quantize an m x n binary32 matrix x (column-major, leading dim ldx) tile
 * by tile.  Tiles are tm x tn blocks anchored at (0, 0); the last row/column
 * of tiles may be partial.  For each tile t: e_t = tile scale exponent of
 * its largest |x|, and q = enc(x * 2^e_t) (exact product in binary64).
 * q is written with leading dimension ldq (elements of 1 or 2 bytes);
 * e is written row-of-tiles fastest: e[ti + tj * ceil(m/tm)].
 */
void oracle_quantize(int fmt, int m, int n, const float *x, int ldx,
                     int tm, int tn, void *q, int ldq, int *e)
{
    int mt = (m + tm - 1) / tm, nt = (n + tn - 1) / tn;
    for (int tj = 0; tj < nt; ++tj)
        for (int ti = 0; ti < mt; ++ti) {
            int i0 = ti * tm, i1 = i0 + tm < m ? i0 + tm : m;
            int j0 = tj * tn, j1 = j0 + tn < n ? j0 + tn : n;
            float amax = 0.0f;
            for (int j = j0; j < j1; ++j)
                for (int i = i0; i < i1; ++i) {
                    float v = fabsf(x[(size_t)i + (size_t)j * ldx]);
                    if (v > amax) amax = v;
                }
            int ex = oracle_tile_scale_exp(fmt, amax);
            e[ti + tj * mt] = ex;
            for (int j = j0; j < j1; ++j)
                for (int i = i0; i < i1; ++i) {
                    float xv = x[(size_t)i + (size_t)j * ldx];
                    size_t o = (size_t)i + (size_t)j * ldq;
                    if (fmt == FMT_BF16)
                        ((uint16_t *)q)[o] = oracle_enc_bf16(xv);
                    else if (fmt == FMT_FP16)
                        ((uint16_t *)q)[o] = oracle_enc_f16(ldexp((double)xv, ex));
                    else
                        ((uint8_t *)q)[o] = oracle_enc_e4m3(ldexp((double)xv, ex));
                }
        }
}
