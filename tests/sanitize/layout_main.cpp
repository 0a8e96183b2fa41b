// Host-side bounds check of the decode kernel's LDS layout (lds_layout in
// grand_internal.h) for every launch shape the host can choose: the next
// power of two of 2L from 1 to 1024, workgroups of 64 to 1024 threads, low
// tables of 2^0 to 2^13 entries.  For each shape it checks that
//   - every region lies inside the layout, and regions that are live at the
//     same time do not overlap;
//   - the overlays of the staging set hold what is built in them: the low
//     table's build buffer and its two subset-XOR tables, and the symbol
//     scores of the cut-off (ni words);
//   - the low table is 8-byte aligned;
//   - the bucket indexes hold nb + 2 entries (nb = keys, read at nb + 1);
//   - the leading-word filter holds 2^filter_log2(b) bits;
//   - the merge of the low table gives each thread at most kMergePer outputs
//     when the host accepts the tuning, and every accepted shape fits in the
//     160 KiB of LDS a compute unit has.
// No GPU is needed.
#include <cstdio>
#include <cstdint>
#include <vector>

#include "grand_internal.h"

using namespace grand;

static int fails = 0;
#define EXPECT(cond, ...)                                                      \
    do {                                                                       \
        if (!(cond)) {                                                         \
            if (fails < 20)                                                    \
                std::printf("failed: %s at ni=%u block=%u b=%u\n", #cond, ni, block, b); \
            fails++;                                                           \
        }                                                                      \
    } while (0)

struct Region {
    const char *name;
    uint32_t off, len;
};

int main()
{
    uint64_t shapes = 0;
    for (uint32_t ni = 1; ni <= kMaxItems; ni <<= 1) {
        for (uint32_t block = 64; block <= kMaxBlock; block += 64) {
            for (uint32_t b = 0; b <= kMaxLowBits; b++) {
                // the host accepts a tuning when each thread merges at most
                // kMergePer outputs and its largest launch (2L = 1024) fits
                // the compute unit's LDS with the static scalars
                if ((1u << b) > kMergePer * block ||
                    4ull * lds_layout(kMaxItems, block, b).words + 256 > 160u * 1024u)
                    continue;
                const LdsLayout L = lds_layout(ni, block, b);
                const uint32_t LB = 1u << b;
                shapes++;
                EXPECT(4ull * L.words + 256 <= 160u * 1024u);
                const uint32_t staging_end = L.iidx;   // the overlays live below it
                std::vector<Region> live = {
                    {"yhat", L.yhat, kMaxN / 32}, {"s0", L.s0, kMaxKW},
                    {"ikey", L.ikey, ni}, {"col0", L.col0, ni},
                    {"lcol", L.lcol, kMaxLowBits * kMaxKW},
                    {"staging", L.foff, staging_end - L.foff},
                    {"iidx", L.iidx, kBucketsPerKey * ni + 2},
                    {"lidx", L.lidx, kBucketsPerKey * LB + 2},
                    {"lkey", L.lkey, LB}, {"ls0", L.ls0, LB},
                    {"lfilt", L.lfilt, 1u << (filter_log2(b) - 5)}};
                for (const Region &r : live)
                    EXPECT(r.off + r.len <= L.words);
                for (size_t i = 0; i < live.size(); i++)
                    for (size_t j = i + 1; j < live.size(); j++) {
                        const Region &x = live[i], &y = live[j];
                        EXPECT(x.off + x.len <= y.off || y.off + y.len <= x.off);
                    }
                // the six per-slot staging arrays, one slot per thread
                const uint32_t st[6] = {L.foff, L.fa, L.fb, L.fcost, L.flead, L.fown};
                for (int k = 0; k < 6; k++) {
                    EXPECT(st[k] >= L.foff && st[k] + block <= staging_end);
                    for (int m = k + 1; m < 6; m++)
                        EXPECT(st[k] + block <= st[m] || st[m] + block <= st[k]);
                }
                // overlays of the staging set: merge buffer, then the subset
                // tables of the table's lower and upper halves behind it
                const uint32_t blo = (b + 1) / 2;
                const uint32_t lt = LB + (1u << blo) + (1u << (b - blo));
                EXPECT(L.ltmp == L.foff);
                EXPECT(L.ltmp + lt <= staging_end);
                EXPECT(L.ltmp + ni <= staging_end);   // the cut-off's symbol scores
                // alignment of the low table
                EXPECT(L.lkey % 2 == 0);
                // the leading-word filter: filt_key takes the word index
                // from hash bits 21-31 at most (fbits - 5 of them), above
                // the bit positions' hash bits 6-20
                EXPECT(filter_log2(b) >= 5 && filter_log2(b) <= 16);
            }
        }
    }
    std::printf("layout check: %llu shapes, %d failures\n", (unsigned long long)shapes, fails);
    return fails != 0;
}
