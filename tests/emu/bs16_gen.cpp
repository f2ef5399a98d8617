// Writes the bit-sliced kernel source that the library generates for a
// GF(2^16) matrix (linked against the library, calling its generator).
// argv: matrix_file source_file.  matrix_file: rows cols (uint32 each), then
// rows x cols uint16 coefficients, row-major.  Exit 3: no source (the matrix
// is over the size limit).  Prints "groups est_ops".
#include <cstdio>
#include <vector>

#include "bitslice.hpp"
#include "gf16.hpp"

int main(int argc, char **argv) {
    if (argc != 3) return 1;
    FILE *f = fopen(argv[1], "rb");
    uint32_t hdr[2];
    if (!f || fread(hdr, 4, 2, f) != 2) return 2;
    pmrc::w16::Mat16 A(static_cast<int>(hdr[0]), static_cast<int>(hdr[1]));
    if (fread(A.v.data(), 2, A.v.size(), f) != A.v.size()) return 2;
    fclose(f);
    std::unique_ptr<pmrc::BsProgram> bp = pmrc::w16::bs16_generate(A);
    printf("%d %ld\n", bp->ngroups, bp->est_ops);
    const std::string &src = bp->k[pmrc::BS_SINGLE].source;
    if (src.empty()) return 3;
    FILE *o = fopen(argv[2], "w");
    if (!o || fputs(src.c_str(), o) < 0) return 4;
    fclose(o);
    return 0;
}
