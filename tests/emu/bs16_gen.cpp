// Writes the bit-sliced kernel source that the library generates for a
// GF(2^16) matrix (linked against the library, calling its generator).
// argv: matrix_file source_file [parts].  matrix_file: rows cols (uint32
// each), then rows x cols uint16 coefficients, row-major.  Without "parts":
// the single kernel, printing "groups est_ops"; exit 3 when there is none
// (the matrix is over the size limit).  With "parts": every part of the
// split form to source_file.part<i>, printing "nparts" and then each part's
// "groups est_ops"; exit 3 when the matrix has no bit-sliced form.
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "bitslice.hpp"
#include "gf16.hpp"

static int write(const std::string &path, const std::string &src) {
    FILE *o = fopen(path.c_str(), "w");
    if (!o || fputs(src.c_str(), o) < 0) return 4;
    fclose(o);
    return 0;
}

int main(int argc, char **argv) {
    if (argc != 3 && !(argc == 4 && !strcmp(argv[3], "parts"))) return 1;
    FILE *f = fopen(argv[1], "rb");
    uint32_t hdr[2];
    if (!f || fread(hdr, 4, 2, f) != 2) return 2;
    pmrc::w16::Mat16 A(static_cast<int>(hdr[0]), static_cast<int>(hdr[1]));
    if (fread(A.v.data(), 2, A.v.size(), f) != A.v.size()) return 2;
    fclose(f);
    if (argc == 4) {
        std::vector<std::unique_ptr<pmrc::BsProgram>> parts = pmrc::w16::bs16_generate_parts(A);
        printf("%zu\n", parts.size());
        for (size_t i = 0; i < parts.size(); ++i) {
            printf("%d %ld\n", parts[i]->ngroups, parts[i]->est_ops);
            if (int rc = write(std::string(argv[2]) + ".part" + std::to_string(i), parts[i]->k[pmrc::BS_SINGLE].source))
                return rc;
        }
        return parts.empty() ? 3 : 0;
    }
    std::unique_ptr<pmrc::BsProgram> bp = pmrc::w16::bs16_generate(A);
    printf("%d %ld\n", bp->ngroups, bp->est_ops);
    const std::string &src = bp->k[pmrc::BS_SINGLE].source;
    if (src.empty()) return 3;
    return write(argv[2], src);
}
