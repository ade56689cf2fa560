// Host build of the line maps of the FFT passes: for a selection of lines
// with fields innermost (the inverse z pass into the field-interleaved grid)
// and the plain field-major selection (the forward z pass), every pass line
// L < lines maps to an in-bounds selection index and an in-bounds element
// range, and the clamp the pass applies to threads past the last line
// (L -> lines - 1) keeps them in bounds too. Prints one line per case:
// name max_sel_index nsel max_first max_last limit.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "fft_map.h"

using namespace aim::fftk;

static void run(const char *name, const ContigMap &m, int64_t lines, int64_t nsel, int64_t n_elem,
                int64_t limit, int tile) {
  int64_t max_sel = -1, max_first = 0, max_last = 0;
  const int64_t blocks = (lines + tile - 1) / tile;
  for (int64_t L0 = 0; L0 < blocks * tile; ++L0) {
    const int64_t L = L0 < lines ? L0 : lines - 1;  // the pass's clamp
    const int64_t s = sel_index(m, L);
    if (s > max_sel) max_sel = s;
    const int64_t b = contig_base(m, L);
    if (b > max_first) max_first = b;
    if (b + (n_elem - 1) * m.es > max_last) max_last = b + (n_elem - 1) * m.es;
  }
  std::printf("%s %lld %lld %lld %lld %lld\n", name, (long long)max_sel, (long long)nsel,
              (long long)max_first, (long long)max_last, (long long)limit);
}

int main() {
  const int64_t Nx = 23, Ny = 19, Nz = 17, Pzs = 48, A1 = Nx * Ny, V1 = A1 * Pzs;
  std::vector<int32_t> sel;
  for (int64_t l = 0; l < A1; l += 3) sel.push_back((int32_t)l);
  const int64_t nl = (int64_t)sel.size();
  for (int64_t F : {4, 8, 64}) {
    char nm[64];
    std::snprintf(nm, sizeof nm, "inner_in_F%lld", (long long)F);
    run(nm, fields_inner(F, V1, Pzs, 1, sel.data(), nl), F * nl, nl, Pzs, F * V1, 14);
    std::snprintf(nm, sizeof nm, "inner_out_F%lld", (long long)F);
    run(nm, fields_inner(F, 1, Nz * F, F, sel.data(), nl), F * nl, nl, Nz, F * A1 * Nz, 14);
    std::snprintf(nm, sizeof nm, "major_in_F%lld", (long long)F);
    run(nm, select_lines(contig_map(Nz), sel.data(), nl, A1), F * nl, nl, Nz, F * A1 * Nz, 14);
  }
  return 0;
}
