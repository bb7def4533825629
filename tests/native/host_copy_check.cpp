// Checks ley::CopyTeam (the external sorts' parallel host copy): copies of
// many sizes, below and above the size where the team splits the work, with
// the team reused between copies; every destination byte must match.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_1909_08006_amd/csrc/host_copy.h"

int main() {
    const size_t sizes[] = {0, 1, 63, 4096, (8u << 20) - 1, 8u << 20, (8u << 20) + 1, 12345677, 33u << 20};
    std::vector<uint8_t> src(33u << 20), dst(33u << 20);
    for (size_t i = 0; i < src.size(); i++) src[i] = (uint8_t)(i * 2654435761u >> 13);
    ley::CopyTeam team;
    for (int round = 0; round < 3; round++) {
        for (size_t n : sizes) {
            std::fill(dst.begin(), dst.end(), (uint8_t)0xA5);
            const size_t off = (size_t)round * 3;  // unaligned starts
            if (n + off > src.size()) continue;
            team.copy(dst.data() + off, src.data() + off, n);
            for (size_t i = 0; i < dst.size(); i++) {
                const uint8_t want = (i >= off && i < off + n) ? src[i] : (uint8_t)0xA5;
                if (dst[i] != want) {
                    std::printf("mismatch: size %zu offset %zu byte %zu\n", n, off, i);
                    return 1;
                }
            }
        }
    }
    std::printf("ok\n");
    return 0;
}
