// Independent Philox4x32-10 reference for the oracle's pin: evaluates
// rocRAND's philox4x32_10 engine (open-source header, run on the host) at
// given counters and keys. Reads lines "c0 c1 c2 c3 k0 k1" (decimal) from
// stdin, prints "w0 w1 w2 w3" per line.
//
// rocRAND's engine initialised at (seed, subsequence, 0) and skipped ahead
// by 4*c numbers sits at the counter (c as 64 bits, subsequence as 64 bits)
// under key (lo seed, hi seed); rocrand4 then returns that block's words.
// The skip is split (four skips of c/4 blocks, then c%4 blocks) so that no
// skip of 4*blocks numbers overflows 64 bits.
#include <rocrand/rocrand_kernel.h>

#include <cstdio>

int main() {
    unsigned long long c0, c1, c2, c3, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = k0 | (k1 << 32);
        unsigned long long subseq = c2 | (c3 << 32);
        unsigned long long c = c0 | (c1 << 32);
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, subseq, 0ull, &st);
        for (int part = 0; part < 4; ++part) skipahead(4ull * (c >> 2), &st);
        skipahead(4ull * (c & 3ull), &st);
        uint4 r = rocrand4(&st);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
