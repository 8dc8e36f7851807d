// Host build of the stochastic-rounding conversions of storage.h (the same
// source the kernels compile), checked exhaustively over the hash bits they
// use: the mean of the rounded values equals the input (unbiased rounding)
// and both neighbouring representable values occur.  Prints one line per
// failure and exits with the number of failures.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "../paper_1410_5584_amd/csrc/storage.h"

using namespace fmlb;

static double half_value(unsigned short b)
{
    return (double)__half2float(__ushort_as_half(b));
}

static double bf16_value(unsigned short b)
{
    const unsigned int u = (unsigned int)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// Mean over every value of the used hash bits; the spacing q of the two
// representable neighbours; the allowed error of the mean is q * 2^-(bits-1)
// (the dither's own resolution) plus FP32 rounding of the input.
static int check(const char *fmt, float v, int bits, double q)
{
    double sum = 0, lo = INFINITY, hi = -INFINITY;
    const unsigned n = 1u << bits;
    for (unsigned k = 0; k < n; ++k) {
        const unsigned int h = k << (32 - bits);
        const double r = fmt[0] == 'b' ? bf16_value(bf16_bits_sr(v, h)) : half_value(f16_bits_sr(v, h));
        sum += r;
        lo = r < lo ? r : lo;
        hi = r > hi ? r : hi;
    }
    const double mean = sum / n;
    const double tol = q * std::ldexp(1.0, 1 - bits) + std::fabs((double)v) * 1e-7;
    int bad = 0;
    if (!(std::fabs(mean - (double)v) <= tol)) {
        std::printf("%s v=%.9g: mean %.12g off by %.3g (tol %.3g)\n", fmt, (double)v, mean, mean - (double)v, tol);
        bad = 1;
    }
    if (!(hi - lo > 0.5 * q && hi - lo < 1.5 * q)) {
        std::printf("%s v=%.9g: neighbours %.9g %.9g, spacing %.3g\n", fmt, (double)v, lo, hi, q);
        bad = 1;
    }
    return bad;
}

int main()
{
    int bad = 0;
    // FP16 subnormals (spacing 2^-24), the smallest normal binade and beyond.
    const float f16v[] = {3.3e-8f, -4.1e-7f, 1.2345e-5f, -2.7e-5f, 6.0e-5f, 6.3e-5f, -1.1e-4f, 3.3e-3f, 0.77f};
    for (float v : f16v) {
        const double a = std::fabs((double)v);
        const double q = a < std::ldexp(1.0, -14) ? std::ldexp(1.0, -24) : std::ldexp(1.0, (int)std::floor(std::log2(a)) - 10);
        bad += check(a < std::ldexp(1.0, -14) ? "f16sub" : "f16", v, a < std::ldexp(1.0, -14) ? 16 : 13, q);
    }
    // BF16 (8 mantissa bits kept, 16 dithered).
    const float bfv[] = {1.2345e-5f, -3.3e-3f, 0.7777f, -1.31f};
    for (float v : bfv) {
        const double q = std::ldexp(1.0, (int)std::floor(std::log2(std::fabs((double)v))) - 7);
        bad += check("bf16", v, 16, q);
    }
    // The hash: every input changes the output (site, value, step, both key words).
    const unsigned h0 = sr_hash(5, 7, 11, 13, 17);
    if (sr_hash(6, 7, 11, 13, 17) == h0 || sr_hash(5, 8, 11, 13, 17) == h0 || sr_hash(5, 7, 12, 13, 17) == h0 ||
        sr_hash(5, 7, 11, 14, 17) == h0 || sr_hash(5, 7, 11, 13, 18) == h0) {
        std::printf("hash ignores an input\n");
        ++bad;
    }
    std::printf(bad ? "FAILED %d\n" : "ok\n", bad);
    return bad;
}
