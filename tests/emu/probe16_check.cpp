// Host check of the probe of the workgroup pivots among the top 2^16 ranks
// (tc_count_mid.hip): bitmap_build, run by an emulated workgroup, against
// the bitmap's definition (word x: bit b for value 32 x + b of the row,
// and the number of row entries before the word), then bitmap16_run on
// random runs of a 16-bit column stream (odd and even starts, full and
// partial runs) against brute force: hit mask bit k for entry c0 + k of
// the run when it lies inside the tail and in the row, and one count per
// hit at the entry's place in the row.  probe16_body.inc is the code of
// the two routines, extracted from tc_count_mid.hip by the test.
#include "hip_cpu.h"

constexpr int BITMAP16_WORDS = 2048;

template <typename T> inline T tc_wave_incl_scan(T x) {
    const int l = __lane_id();
    for (int off = 1; off < TC_WAVE; off <<= 1) {
        const T y = __shfl_up(x, (unsigned)off, TC_WAVE);
        if (l >= off) x += y;
    }
    return x;
}

#include "probe16_body.inc"

static uint64_t rs_ = 99;
static uint64_t rnd() {
    rs_ ^= rs_ << 13;
    rs_ ^= rs_ >> 7;
    rs_ ^= rs_ << 17;
    return rs_;
}

int main() {
    int fails = 0;
    const int32_t r16 = 1000000;  // the rank the 16-bit values start from
    for (int trial = 0; trial < 6; ++trial) {
        // the pivot's row: d distinct values in [1, 65536), sorted, as ranks
        const int d = trial == 0 ? 1 : trial == 1 ? 2000 : 1 + (int)(rnd() % 1800);
        std::vector<int> vals;
        std::vector<char> in(65536, 0);
        while ((int)vals.size() < d) {
            const int x = 1 + (int)(rnd() % 65535);
            if (!in[x]) {
                in[x] = 1;
                vals.push_back(x);
            }
        }
        std::sort(vals.begin(), vals.end());
        std::vector<int> place(65536, -1);
        for (int j = 0; j < d; ++j) place[vals[j]] = j;
        const int64_t vstart = 5;
        std::vector<int32_t> ocol(vstart + d + 8, 0);
        for (int j = 0; j < d; ++j) ocol[vstart + j] = r16 + vals[j];
        std::vector<uint2> bm(BITMAP16_WORDS, uint2{0xDEADBEEFu, 0xDEADBEEFu});
        std::vector<uint32_t> scan(16);
        uint2 *bp = bm.data();
        uint32_t *sp = scan.data();
        const int32_t *op = ocol.data();
        emu_launch(1, 256, [=]() { bitmap_build(bp, sp, op, vstart, d, (uint32_t)r16, 32u * BITMAP16_WORDS); });
        int64_t bad_bm = 0;
        uint32_t before = 0;
        for (int x = 0; x < BITMAP16_WORDS; ++x) {
            uint32_t bits = 0;
            for (int b = 0; b < 32; ++b) bits |= (uint32_t)in[32 * x + b] << b;
            bad_bm += bm[x].x != bits || bm[x].y != before;
            before += (uint32_t)__builtin_popcount(bits);
        }
        // a 16-bit column stream: row values, other values, and 0 (ranks
        // below r16), with 64 entries of padding
        const int64_t N = 20000;
        std::vector<uint16_t> col(N + 64, 0);
        for (int64_t k = 0; k < N; ++k) {
            const uint64_t c = rnd() % 10;
            col[k] = c < 4 ? (uint16_t)vals[rnd() % d] : c < 9 ? (uint16_t)(rnd() % 65536) : 0;
        }
        int64_t bad_mask = 0, bad_cnt = 0, runs = 0;
        std::vector<uint32_t> lsup(d + 64), want(d + 64);
        for (int r = 0; r < 3000; ++r) {
            const int64_t c0 = (int64_t)(rnd() % (N - 32));
            const int cnt = r % 3 == 0 ? 32 : 1 + (int)(rnd() % 32);
            std::fill(lsup.begin(), lsup.end(), 0u);
            std::fill(want.begin(), want.end(), 0u);
            uint32_t wmask = 0;
            for (int k = 0; k < cnt; ++k) {
                const int p = place[col[c0 + k]];
                if (p >= 0) {
                    wmask |= 1u << k;
                    want[p] += 1;
                }
            }
            const uint32_t mask = bitmap16_run(col.data(), c0, cnt, bm.data(), lsup.data());
            bad_mask += mask != wmask;
            bad_cnt += lsup != want;
            ++runs;
        }
        printf("row of %d entries: bitmap mismatches %lld; %lld runs, mask mismatches %lld, "
               "count mismatches %lld\n", d, (long long)bad_bm, (long long)runs,
               (long long)bad_mask, (long long)bad_cnt);
        fails += bad_bm != 0 || bad_mask != 0 || bad_cnt != 0;
    }
    return fails ? 1 : 0;
}
