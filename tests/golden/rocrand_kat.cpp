// Known-answer vectors for Philox4x32-10 taken from rocRAND's own engine
// (a third-party implementation of the published generator), run on the host.
// Counter (c0, c1, c2, c3) maps to rocRAND's state as subsequence = c2 | c3 << 32
// and offset = 4 * (c0 | c1 << 32) (so c1 < 2^30 here); key (k0, k1) = seed lo / hi.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdint>

int main() {
    // fixed, spread-out inputs (no randomness needed to choose them)
    const uint32_t cases[][6] = {
        {0u, 0u, 0u, 0u, 0u, 0u},
        {0xffffffffu, 0x3fffffffu, 0xffffffffu, 0xffffffffu, 0xffffffffu, 0xffffffffu},
        {0x243f6a88u, 0x05a308d3u, 0x13198a2eu, 0x03707344u, 0xa4093822u, 0x299f31d0u},
        {1u, 2u, 3u, 4u, 0u, 0u},
        {4095u, 0u, 3u, 1u, 0u, 0u},
        {262143u, 15u, 8u, 1u, 0u, 0u},
        {12345u, 7u, 2u, 0u, 0u, 1u},
        {77u, 0u, 0u, 0u, 42u, 7u},
    };
    for (const auto &c : cases) {
        unsigned long long seed = (unsigned long long)c[4] | ((unsigned long long)c[5] << 32);
        unsigned long long subseq = (unsigned long long)c[2] | ((unsigned long long)c[3] << 32);
        unsigned long long offset = 4ull * ((unsigned long long)c[0] | ((unsigned long long)c[1] << 32));
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, subseq, offset, &st);
        uint4 r = rocrand4(&st);
        std::printf("%u %u %u %u %u %u %u %u %u %u\n", c[0], c[1], c[2], c[3], c[4], c[5], r.x, r.y, r.z, r.w);
    }
    return 0;
}
