// Host check of the fold kernels (k_fold, k_fold_big) of tc_count_mid.hip
// on the CPU emulation: random triangular bit matrices B_u (row i of a row
// with d entries holds d - 1 - i bits, bit b <-> column i + 1 + b, padded
// rows as the count writes them) folded into supports that start at random
// values, against brute force: every set bit adds 1 to its row's slot and
// to its column's slot.  fold_body.inc is the kernels' source, extracted
// from tc_count_mid.hip by the test.
#include "hip_cpu.h"
#include "fold_body.inc"

static uint64_t rs_ = 12345;
static uint64_t rnd() {
    rs_ ^= rs_ << 13;
    rs_ ^= rs_ >> 7;
    rs_ ^= rs_ << 17;
    return rs_;
}

struct Case {
    std::vector<int64_t> orp, rowbase;
    std::vector<uint32_t> bits, sup, want;
    std::vector<int32_t> rows;
};

// rows of the given lengths and bit densities; 4 words of padding after
// the last row, as the library allocates them
static Case make(const std::vector<int64_t> &d, const std::vector<double> &p) {
    Case c;
    const int64_t R = (int64_t)d.size();
    c.orp.assign(R + 1, 0);
    c.rowbase.assign(R + 1, 0);
    for (int64_t r = 0; r < R; ++r) {
        c.orp[r + 1] = c.orp[r] + d[r];
        c.rowbase[r + 1] = c.rowbase[r] + bit_words(d[r]);
    }
    c.bits.assign(c.rowbase[R] + 4, 0);
    c.sup.resize(c.orp[R]);
    for (auto &x : c.sup) x = (uint32_t)(rnd() & 0xFFFF);
    c.want = c.sup;
    for (int64_t r = 0; r < R; ++r) {
        int64_t off = c.rowbase[r];
        for (int64_t i = 0; i + 1 < d[r]; ++i) {
            const int64_t len = d[r] - 1 - i;
            for (int64_t b = 0; b < len; ++b)
                if ((double)(rnd() % 1000000) < p[r] * 1000000.0) {
                    c.bits[off + b / 32] |= 1u << (b % 32);
                    c.want[c.orp[r] + i] += 1;
                    c.want[c.orp[r] + i + 1 + b] += 1;
                }
            off += (len + 31) / 32;
        }
    }
    c.rows.resize(R);
    for (int64_t r = 0; r < R; ++r) c.rows[r] = (int32_t)r;
    return c;
}

static int report(const char *what, const Case &c) {
    int64_t bad = 0;
    for (size_t k = 0; k < c.sup.size(); ++k) bad += c.sup[k] != c.want[k];
    printf("%s: %zu rows, %zu slots, %lld mismatches\n", what, c.rows.size(), c.sup.size(),
           (long long)bad);
    return bad != 0;
}

int main() {
    int fails = 0;
    const std::vector<int64_t> big = {65, 70, 96, 97, 100, 128, 129, 200, 300, 511, 512,
                                      600, 1000, 1023, 1024, 1025, 1500, 2047, 2048, 2049,
                                      2100, 3000};
    const double dens[] = {1.0, 0.5, 0.05};  // 1.0: the largest counts
    // big rows: 32-bit kernel (private partials up to 1024 entries, one
    // owner or atomics above), 64-bit kernel, and LDS counters smaller than
    // some rows (those add to the support by atomic)
    for (int mode = 0; mode < 3; ++mode) {
        std::vector<int64_t> d;
        std::vector<double> p;
        for (double q : dens)
            for (int64_t x : big) {
                d.push_back(x);
                p.push_back(q);
            }
        Case c = make(d, p);
        int dcap = (int)std::min<int64_t>(*std::max_element(d.begin(), d.end()), 7936);
        if (mode == 2) dcap = 1000;
        dcap = (dcap + 3) & ~3;
        const int64_t i32 = mode == 1 ? 0 : FOLD_I32_MAX;
        std::vector<uint32_t> lds(4 * fold_wave_words(dcap));
        colc_lds = lds.data();
        const int32_t *rp = c.rows.data();
        const int64_t *op = c.orp.data(), *rb = c.rowbase.data();
        const uint32_t *bp = c.bits.data();
        uint32_t *sp = c.sup.data();
        const int64_t R = (int64_t)c.rows.size();
        emu_launch(2, 256, [=]() { k_fold_big<int32_t>(rp, R, op, rb, bp, sp, dcap, i32); });
        emu_launch(2, 256, [=]() { k_fold_big<int64_t>(rp, R, op, rb, bp, sp, dcap, i32); });
        const char *name[] = {"big rows, 32-bit", "big rows, 64-bit", "big rows, small LDS cap"};
        fails += report(name[mode], c);
    }
    {   // rows of 2..64 entries (k_fold<16>); a multiple of the 32 groups of
        // the launch, so that every emulated lane reaches the same shuffles
        std::vector<int64_t> d;
        std::vector<double> p;
        for (double q : dens)
            for (int64_t x = 2; x <= 64; ++x) {
                d.push_back(x);
                p.push_back(q);
            }
        while (d.size() % 32) {
            d.push_back(2 + (int64_t)(rnd() % 63));
            p.push_back(0.3);
        }
        Case c = make(d, p);
        const int32_t *rp = c.rows.data();
        const int64_t *op = c.orp.data(), *rb = c.rowbase.data();
        const uint32_t *bp = c.bits.data();
        uint32_t *sp = c.sup.data();
        const int64_t R = (int64_t)c.rows.size();
        emu_launch(2, 256, [=]() { k_fold<16>(rp, R, op, rb, bp, sp); });
        fails += report("small rows", c);
    }
    return fails ? 1 : 0;
}
