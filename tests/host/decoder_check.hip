// Host build of the library's block decoders (the device header compiled for
// the CPU), checked value for value against the oracle's decoder on random
// block bits at every rate: the plain plane-by-plane decoder for both
// precisions, the two-pass decoders of both precisions over an emulated
// LDS staging area (one lane's view; the row past the block's words holds
// garbage, as the next row or the record area does on the GPU), and the
// low-rate double-precision decoder (the blocks it takes; it must leave the
// others untouched).
// Exit status 0 iff every value matches bit for bit.
#include "../../paper_2009_03254_amd/csrc/zfp_device.h"

#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

extern "C" int oracle_zfp_decode_some(const uint64_t *stream, int is_f64, uint32_t rate,
                                      const uint32_t *ids, uint64_t n, float *blocks);

int main() {
    std::mt19937_64 rng(12345);
    long bad = 0, total = 0, low_taken = 0, low_back = 0;
    const int rates[] = {1, 2, 3, 4, 5, 6, 7, 8, 9, 12, 16, 24, 32};
    const double dens[] = {0.5, 0.2, 0.05, 0.01, 0.9, 0.7};
    const int ext64[] = {-1000, -300, -127, -126, -121, -110, -97, -96, 96, 97, 126, 127, 300, 900};
    const int ext32[] = {-126, -110, -100, -97, -96, 96, 97, 100, 127};
    for (int f64 = 0; f64 < 2; f64++)
        for (int rate : rates)
            for (double p : dens) {
                const int nb = 1500;
                std::vector<uint64_t> s((size_t)nb * rate);
                std::bernoulli_distribution B(p);
                const int eb = f64 ? 11 : 8, bias = f64 ? 1023 : 127;
                for (int b = 0; b < nb; b++) {
                    for (int w = 0; w < rate; w++) {
                        uint64_t v = 0;
                        for (int i = 0; i < 64; i++) v |= (uint64_t)B(rng) << i;
                        s[(size_t)b * rate + w] = v;
                    }
                    // nonzero flag and an exponent near 0; every 11th block one near
                    // the ends of the range (values beyond single precision, either
                    // way, and both sides of the single-precision scale's range)
                    uint64_t &w0 = s[(size_t)b * rate];
                    int eo = -20 + (int)(rng() % 41);
                    if (b % 11 == 5) eo = f64 ? ext64[rng() % 14] : ext32[rng() % 9];
                    const uint64_t e = (uint64_t)(bias + eo);
                    w0 = (w0 & ~((1ull << (eb + 1)) - 1)) | 1ull | (e << 1);
                    if (b % 97 == 0) w0 &= ~1ull;   // some all-zero blocks
                }
                std::vector<uint32_t> ids(nb);
                for (int b = 0; b < nb; b++) ids[b] = (uint32_t)b;
                std::vector<float> ref((size_t)nb * 64), got((size_t)nb * 64);
                if (oracle_zfp_decode_some(s.data(), f64, rate, ids.data(), nb, ref.data()) != 0) {
                    printf("oracle decode failed\n");
                    return 2;
                }
                for (int b = 0; b < nb; b++) {
                    if (f64) bcmc::decode_block<true>(s.data() + (size_t)b * rate, rate, got.data() + (size_t)b * 64);
                    else bcmc::decode_block<false>(s.data() + (size_t)b * rate, rate, got.data() + (size_t)b * 64);
                }
                long n1 = 0, n2 = 0;
                for (size_t i = 0; i < got.size(); i++) n1 += memcmp(&got[i], &ref[i], 4) != 0;
                if (rate <= bcmc::STAGE_MAX_RATE) {
                    std::vector<uint64_t> st((size_t)bcmc::STAGE_STRIDE * (rate + 1), 0x5A5A5A5A5A5A5A5Aull);
                    uint32_t rec[bcmc::RecLayout<true>::STRIDE];
                    for (int b = 0; b < nb; b++) {
                        for (int w = 0; w < rate; w++) st[(size_t)w * bcmc::STAGE_STRIDE] = s[(size_t)b * rate + w];
                        for (auto &r : rec) r = 0xDEADBEEFu;   // written before read
                        if (f64) bcmc::decode_block_staged_f64(st.data(), rec, rate, got.data() + (size_t)b * 64);
                        else bcmc::decode_block_staged_f32(st.data(), rec, rate, got.data() + (size_t)b * 64);
                    }
                    for (size_t i = 0; i < got.size(); i++) n2 += memcmp(&got[i], &ref[i], 4) != 0;
                    if (f64) {   // the low-rate decoder: the blocks it takes, value for value
                        for (int b = 0; b < nb; b++) {
                            for (int w = 0; w < rate; w++) st[(size_t)w * bcmc::STAGE_STRIDE] = s[(size_t)b * rate + w];
                            for (auto &r : rec) r = 0xDEADBEEFu;
                            float *o = got.data() + (size_t)b * 64;
                            for (int i = 0; i < 64; i++) o[i] = -1.0f;
                            if (bcmc::decode_block_staged_f64_low(st.data(), rec, rate, o)) {
                                low_taken++;
                                for (int i = 0; i < 64; i++) n2 += memcmp(&o[i], &ref[(size_t)b * 64 + i], 4) != 0;
                            } else {
                                low_back++;
                                for (int i = 0; i < 64; i++) n2 += o[i] != -1.0f;   // untouched
                            }
                        }
                    }
                }
                total += nb;
                if (n1 || n2)
                    printf("f64=%d rate=%d density=%.2f: %ld (plain) %ld (two-pass) mismatching values\n", f64,
                           rate, p, n1, n2);
                bad += n1 + n2;
            }
    printf("low-rate decoder: %ld blocks decoded, %ld handed back\n", low_taken, low_back);
    printf("blocks %ld, mismatching values %ld\n", total, bad);
    return bad != 0 || low_taken < 10000 || low_back < 10000;
}
