// Host replay of particle states through the index arithmetic of the GPU kernels
// (paper_2002_08855_amd/csrc/index_math.h, the same functions the kernels call): every
// node a point's delta-function support reaches (Eqs. 47-48) must lie inside its LDS box
// and inside the lattice, and be within the kernel's reach of the point; cell
// coordinates (Eqs. 49-51), the pair-search window and the interior-momentum box must stay
// inside their arrays.  Built for the host with AddressSanitizer and UndefinedBehavior-
// Sanitizer (float-cast-overflow included), so that a conversion of an out-of-range or
// NaN position to int fails the run as well.
//
// Input (text, whitespace separated):
//   dim n0 n1 n2 kind cap nc0 nc1 nc2 invh0 invh1 invh2
//   nstates, then per state: np, then per particle: X0 X1 X2 R nl and nl offsets (x y z)
// Output: "checked <supports> <nodes> <skipped boxes>" and exit 0, or a message and exit 1.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "../paper_2002_08855_amd/csrc/index_math.h"

static long long g_nodes = 0, g_supports = 0, g_skipped = 0;

#define CHECK(cond, ...)                     \
  do {                                       \
    if (!(cond)) {                           \
      fprintf(stderr, "FAIL %s: ", #cond);   \
      fprintf(stderr, __VA_ARGS__);          \
      fprintf(stderr, "\n");                 \
      exit(1);                               \
    }                                        \
  } while (0)

template <int DIM>
static void check_unit(const MarkerGeo& g, int cap, const double* Xc, const double* rlo,
                       const double* rhi, const std::vector<double>& off, int k0, int k1) {
  const PBox<DIM> b = range_box<DIM>(Xc, rlo, rhi, g.kind);
  CHECK(b.n >= 1, "box of %d nodes", b.n);
  for (int d = 0; d < 3; d++) CHECK(b.B[d] >= 1, "box side %d on axis %d", b.B[d], d);
  if (b.n > cap) {  // the kernels return for such a unit
    g_skipped++;
    return;
  }
  const double reach = g.kind == 0 ? 2.0 : 1.5;
  for (int k = k0; k < k1; k++) {
    double X[3];
    for (int d = 0; d < 3; d++) X[d] = d < DIM ? Xc[d] + off[3 * k + d] : 0.0;
    PointWeights<double> pw;
    point_weights<DIM, double>(g.kind, X, pw);
    g_supports++;
    visit_support<DIM, double>(g, b, pw, [&](int loc, double) {
      CHECK(loc >= 0 && loc < b.n, "box node %d of %d", loc, b.n);
      CHECK(loc < 65536, "box node %d does not fit the uint16 lists", loc);
      int x, y, z;
      b.at(loc, x, y, z);
      const int c[3] = {x, y, z};
      for (int d = 0; d < DIM; d++) {
        CHECK(c[d] >= 0 && c[d] < g.n[d], "node %d %d %d outside the lattice", x, y, z);
        CHECK(fabs(double(c[d]) - X[d]) <= reach, "node %d on axis %d beyond the support of %.17g",
              c[d], d, X[d]);
      }
      if (DIM == 2) CHECK(z == 0, "2-D node with z = %d", z);
      const long long i = x + (long long)g.n[0] * (y + (long long)g.n[1] * z);
      CHECK(i >= 0 && i < (long long)g.n[0] * g.n[1] * g.n[2], "node index %lld", i);
      CHECK((x >> 5) < (g.n[0] + 31) / 32, "bitmap word %d", x >> 5);
      g_nodes++;
    });
    // the point-wise kernels: one lane per support node
    for (int l = 0; l < (DIM == 3 ? 64 : 16); l++) {
      double w;
      bool tr;
      const int i = support_node<DIM, double>(g, X, l, w, tr);
      CHECK(i >= -1 && i < g.n[0] * g.n[1] * g.n[2], "point-wise node %d", i);
    }
  }
}

template <int DIM>
static void check_particle(const MarkerGeo& g, int cap, const int* nc, const double* invh,
                           const double* Xc, double R, const std::vector<double>& off, int nl) {
  // the whole particle, then two runs of its points with their own offset ranges (the
  // split of the work-unit plan)
  {
    const double rlo[3] = {-R, -R, -R}, rhi[3] = {R, R, R};
    check_unit<DIM>(g, cap, Xc, rlo, rhi, off, 0, nl);
  }
  for (int h = 0; h < 2 && nl >= 2; h++) {
    const int k0 = h == 0 ? 0 : nl / 2, k1 = h == 0 ? nl / 2 : nl;
    double rlo[3] = {0, 0, 0}, rhi[3] = {0, 0, 0};
    for (int d = 0; d < 3; d++) {
      rlo[d] = 1e300;
      rhi[d] = -1e300;
      for (int k = k0; k < k1; k++) {
        rlo[d] = fmin(rlo[d], off[3 * k + d]);
        rhi[d] = fmax(rhi[d], off[3 * k + d]);
      }
    }
    check_unit<DIM>(g, cap, Xc, rlo, rhi, off, k0, k1);
  }
  // cells and the 5^d pair-search window
  for (int d = 0; d < DIM; d++) {
    const int c = cell_coord(Xc[d], invh[d], nc[d]);
    CHECK(c >= 0 && c < nc[d], "cell %d of %d", c, nc[d]);
    const int lo = c - 2 > 0 ? c - 2 : 0, hi = c + 2 < nc[d] - 1 ? c + 2 : nc[d] - 1;
    CHECK(lo <= hi && hi < nc[d], "window %d..%d", lo, hi);
  }
  // interior momentum box
  int lo[3], hi[3];
  interior_box(Xc, R, g.n, DIM, lo, hi);
  long long total = 1;
  for (int d = 0; d < DIM; d++) {
    CHECK(lo[d] >= 0 && hi[d] <= g.n[d] - 1, "interior box %d..%d on axis %d", lo[d], hi[d], d);
    total *= hi[d] >= lo[d] ? (long long)(hi[d] - lo[d] + 1) : 0;
  }
  CHECK(total <= (long long)g.n[0] * g.n[1] * g.n[2], "interior box of %lld nodes", total);
}

int main(int argc, char** argv) {
  if (argc != 2) {
    fprintf(stderr, "usage: %s states.txt\n", argv[0]);
    return 2;
  }
  FILE* fp = fopen(argv[1], "r");
  if (!fp) return 2;
  MarkerGeo g;
  int cap, nc[3];
  double invh[3];
  if (fscanf(fp, "%d %d %d %d %d %d %d %d %d %lf %lf %lf", &g.dim, &g.n[0], &g.n[1], &g.n[2],
             &g.kind, &cap, &nc[0], &nc[1], &nc[2], &invh[0], &invh[1], &invh[2]) != 12)
    return 2;
  for (int d = 0; d < 3; d++) g.periodic[d] = 0;
  g.width = g.kind == 0 ? 4 : 3;
  int nstates = 0;
  if (fscanf(fp, "%d", &nstates) != 1) return 2;
  for (int s = 0; s < nstates; s++) {
    int np = 0;
    if (fscanf(fp, "%d", &np) != 1) return 2;
    for (int p = 0; p < np; p++) {
      double Xc[3], R;
      int nl;
      if (fscanf(fp, "%lf %lf %lf %lf %d", &Xc[0], &Xc[1], &Xc[2], &R, &nl) != 5) return 2;
      std::vector<double> off(3 * (size_t)nl);
      for (int k = 0; k < 3 * nl; k++)
        if (fscanf(fp, "%lf", &off[k]) != 1) return 2;
      if (g.dim == 2)
        check_particle<2>(g, cap, nc, invh, Xc, R, off, nl);
      else
        check_particle<3>(g, cap, nc, invh, Xc, R, off, nl);
    }
  }
  fclose(fp);
  printf("checked %lld %lld %lld\n", g_supports, g_nodes, g_skipped);
  return 0;
}
