// CPU build of the projector's tracer core for the host-side tests: the
// boundary tables (make_tables) and the per-ray walk (core::Walker) exactly
// as the GPU kernels run them, compiled for the host (with AddressSanitizer
// and UndefinedBehaviorSanitizer in the tests, so that every table read is
// bounds-checked).
//
// Usage: walk_cpu IN OUT
//   IN  (little-endian): int32 nr, ne, na; int64 R; float64 r_b[nr+1],
//       e_b[ne+1], a_b[na+1]; float64 starts[R][3], dirs[R][3] (any length)
//   OUT: int32 counts[R]; int32 vox[S]; float64 len[S]; int32 events[R]
//       (crossing events processed per ray), S = sum of counts
// The directions are normalised as tsp_geometry_create does for explicit
// rays.  Exit status 0 on success, 2 on a malformed input.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "tsp_trace_core.h"

using namespace tsp;
using namespace tsp::core;

template <class T>
static bool rd(FILE *f, T *p, size_t n) {
    return std::fread(p, sizeof(T), n, f) == n;
}

int main(int argc, char **argv) {
    if (argc != 3) {
        std::fprintf(stderr, "usage: walk_cpu IN OUT\n");
        return 2;
    }
    FILE *in = std::fopen(argv[1], "rb");
    if (!in) return 2;
    int32_t sh[3];
    int64_t R;
    if (!rd(in, sh, 3) || !rd(in, &R, 1) || sh[0] < 1 || sh[1] < 1 || sh[2] < 1 || R < 0)
        return 2;
    const int nr = sh[0], ne = sh[1], na = sh[2];
    std::vector<double> rb(nr + 1), eb(ne + 1), ab(na + 1), st(3 * R), dr(3 * R);
    if (!rd(in, rb.data(), rb.size()) || !rd(in, eb.data(), eb.size()) ||
        !rd(in, ab.data(), ab.size()) || !rd(in, st.data(), st.size()) ||
        !rd(in, dr.data(), dr.size()))
        return 2;
    std::fclose(in);

    TabDesc D;
    std::vector<double> tabv;
    make_tables(rb.data(), nr, eb.data(), ne, ab.data(), na, &D, &tabv);
    // the tables in a heap block of exactly n_tab doubles, so that any read
    // past them is a sanitizer error
    double *tab = static_cast<double *>(std::malloc(sizeof(double) * tabv.size()));
    for (size_t i = 0; i < tabv.size(); i++) tab[i] = tabv[i];
    const Tab T = make_tab(D, tab);

    std::vector<int32_t> counts(R), events(R), vox;
    std::vector<double> len;
    for (int64_t i = 0; i < R; i++) {
        const double *s = &st[3 * i], *d = &dr[3 * i];
        const double dn = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const V3 x = {s[0], s[1], s[2]};
        const V3 n = {d[0] / dn, d[1] / dn, d[2] / dn};
        Walker w;
        int c = 0, ev = 0;
        if (w.init(T, x, n)) {
            int v;
            double l;
            while (!w.done()) {
                ev++;
                if (w.step(T, v, l)) {
                    if (v < 0 || v >= nr * ne * na) {
                        std::fprintf(stderr, "ray %lld: voxel %d out of range\n", (long long)i, v);
                        return 3;
                    }
                    vox.push_back(v);
                    len.push_back(l);
                    c++;
                }
            }
        }
        counts[i] = c;
        events[i] = ev;
    }
    std::free(tab);
    FILE *out = std::fopen(argv[2], "wb");
    if (!out) return 2;
    std::fwrite(counts.data(), sizeof(int32_t), counts.size(), out);
    std::fwrite(vox.data(), sizeof(int32_t), vox.size(), out);
    std::fwrite(len.data(), sizeof(double), len.size(), out);
    std::fwrite(events.data(), sizeof(int32_t), events.size(), out);
    std::fclose(out);
    return 0;
}
