// Reference Philox4x32-10 outputs from rocRAND's header implementation, run
// on the host.  Reads lines "key_lo key_hi c0 c1 c2 c3" (decimal) on stdin and
// prints the four output words per line.  rocRAND places the 64-bit seed in
// the key and (offset / 4) in counter words 0-1, the subsequence in words 2-3.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
    unsigned long long klo, khi, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &klo, &khi, &c0, &c1, &c2, &c3) == 6) {
        rocrand_state_philox4x32_10 st;
        const unsigned long long seed = klo | (khi << 32);
        const unsigned long long subseq = c2 | (c3 << 32);
        const unsigned long long offset = 4ULL * (c0 | (c1 << 32));
        rocrand_init(seed, subseq, offset, &st);
        uint4 v = rocrand4(&st);
        std::printf("%u %u %u %u\n", v.x, v.y, v.z, v.w);
    }
    return 0;
}
