// Prints Philox4x32-10 of the counter and key given on the command line
// (six hexadecimal words: c0 c1 c2 c3 k0 k1), computed on the host by the
// library's own generator.
#include <cstdio>
#include <cstdlib>

#include "../paper_1302_1861_amd/csrc/common.hpp"

int main(int argc, char **argv) {
    if (argc != 7) return 2;
    uint32_t v[6];
    for (int i = 0; i < 6; ++i)
        v[i] = (uint32_t)std::strtoul(argv[i + 1], nullptr, 16);
    const psl::u32x4 r =
        psl::philox4x32_10(psl::u32x4{v[0], v[1], v[2], v[3]}, v[4], v[5]);
    std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    return 0;
}
