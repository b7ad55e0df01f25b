// Exhaustive-ish check of the magic-number division used by the layout
// program: floor(n / d) for random and adversarial (n, d) with n < 2^63.
#include <cstdio>
#include <random>

#include "../../paper_2402_12274_amd/csrc/layout_dev.h"

int main()
{
    std::mt19937_64 g(12345);
    long bad = 0, checked = 0;
    auto check = [&](uint64_t n, uint64_t d) {
        mdt::MagicDiv m = mdt::make_magic(d);
        uint64_t q = mdt::magic_div(n, m);
        checked++;
        if (q != n / d) {
            if (bad < 10) std::printf("bad n=%llu d=%llu got %llu want %llu\n", (unsigned long long)n,
                                      (unsigned long long)d, (unsigned long long)q, (unsigned long long)(n / d));
            bad++;
        }
    };
    const uint64_t top = ((uint64_t)1 << 63) - 1;
    for (uint64_t d = 1; d < 3000; d++) {
        for (uint64_t k = 0; k < 64; k++) {
            uint64_t n = d * k;
            check(n, d);
            if (n) check(n - 1, d);
            check(n + 1, d);
        }
        check(top, d);
        check(top - d, d);
        for (int i = 0; i < 50; i++) check(g() & top, d);
    }
    for (int i = 0; i < 2000000; i++) {
        int bits = 1 + (int)(g() % 63);
        uint64_t d = (g() & (((uint64_t)1 << bits) - 1)) | 1;
        uint64_t n = g() & top;
        check(n, d);
        uint64_t k = n / d;
        check(k * d, d);
        if (k) check(k * d - 1, d);
    }
    for (int s = 0; s < 63; s++) {
        uint64_t d = (uint64_t)1 << s;
        check(top, d);
        check(d, d);
        check(d - 1, d);
        check(d + 1, d);
        check(top, d + 1);
        check(top, d - 1 ? d - 1 : 1);
    }
    // 32-bit variant: n < 2^31, 1 <= d < 2^31
    auto check32 = [&](uint32_t n, uint32_t d) {
        mdt::MagicDiv32 m = mdt::make_magic32(d);
        uint32_t q = mdt::magic_div32(n, m);
        checked++;
        if (q != n / d) {
            if (bad < 10) std::printf("bad32 n=%u d=%u got %u want %u\n", n, d, q, n / d);
            bad++;
        }
    };
    const uint32_t top32 = 0x7fffffffu;
    for (uint32_t d = 1; d < 5000; d++) {
        for (uint32_t k = 0; k < 40; k++) {
            uint64_t n = (uint64_t)d * k;
            if (n > top32) break;
            check32((uint32_t)n, d);
            if (n) check32((uint32_t)n - 1, d);
            if (n < top32) check32((uint32_t)n + 1, d);
        }
        check32(top32, d);
        for (int i = 0; i < 40; i++) check32((uint32_t)(g() & top32), d);
    }
    for (int i = 0; i < 2000000; i++) {
        uint32_t d = (uint32_t)(g() % top32) + 1;
        uint32_t n = (uint32_t)(g() & top32);
        check32(n, d);
        uint32_t k = n / d;
        check32(k * d, d);
        if (k) check32(k * d - 1, d);
    }
    std::printf("checked %ld bad %ld\n", checked, bad);
    return bad != 0;
}
