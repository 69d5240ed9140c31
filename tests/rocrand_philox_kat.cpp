// Prints rocRAND's Philox4x32-10 output block for (seed, counter) tuples read
// from stdin, one tuple per line: seed c q mode (decimal).  rocRAND's engine
// starts from counter (0,0,0,0); discard_subsequence(s) adds s to counter words
// 2-3 and an offset of 4c adds c to words 0-1, so the first four outputs are
// the Philox block at counter (c mod 2^32, c >> 32, q, mode) with key (c < 2^62)
// (seed mod 2^32, seed >> 32).  Used only to pin the oracle's Philox.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_kernel.h>
#include <cstdio>

int main() {
    unsigned long long seed, c, q, mode;
    while (std::scanf("%llu %llu %llu %llu", &seed, &c, &q, &mode) == 4) {
        rocrand_device::philox4x32_10_engine e(seed, q | (mode << 32), 4ULL * c);
        unsigned w0 = e(), w1 = e(), w2 = e(), w3 = e();
        std::printf("%u %u %u %u\n", w0, w1, w2, w3);
    }
    return 0;
}
