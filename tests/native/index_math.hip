// Host check of the library's node-index arithmetic (nbr, div_extent) against
// a direct definition: neighbour r + d of every node of small boxes with every
// combination of periodic axes, and t / n over extents up to 2^30.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>
#include "elbm.h"
#include "../../paper_1612_05404_amd/csrc/elbm_device.h"

static int direct_nbr(const elbm::BoxDev &B, int x, int y, int z, int dx, int dy, int dz) {
  const int c[3] = {x + dx, y + dy, z + dz}, n[3] = {B.nx, B.ny, B.nz};
  int w[3];
  for (int a = 0; a < 3; ++a) {
    if (c[a] >= 0 && c[a] < n[a]) w[a] = c[a];
    else if (B.per[a]) w[a] = (c[a] % n[a] + n[a]) % n[a];
    else return -1;
  }
  return w[0] + n[0] * (w[1] + n[1] * w[2]);
}

int main() {
  long checked = 0, bad = 0;
  const int sizes[] = {1, 2, 3, 5, 8};
  for (int a : sizes) for (int b : sizes) for (int c : sizes) for (int per = 0; per < 8; ++per) {
    elbm::BoxDev B{};
    B.nx = a; B.ny = b; B.nz = c;
    for (int k = 0; k < 3; ++k) B.per[k] = (per >> k) & 1;
    for (int z = 0; z < c; ++z) for (int y = 0; y < b; ++y) for (int x = 0; x < a; ++x)
      for (int dz = -1; dz <= 1; ++dz) for (int dy = -1; dy <= 1; ++dy) for (int dx = -1; dx <= 1; ++dx) {
        ++checked;
        if (elbm::nbr(B, x, y, z, dx, dy, dz) != direct_nbr(B, x, y, z, dx, dy, dz)) ++bad;
      }
  }
  srand(7);
  for (int n = 1; n <= 20000; ++n) {
    const double rn = 1.0 / n;
    const long kmax = (1L << 30) / n;
    for (int j = 0; j < 24; ++j) {
      long k = j < 12 ? j : (long)(kmax * (double)rand() / RAND_MAX);
      const long ts[3] = {k * n - 1, k * n, k * n + n - 1};
      for (long t : ts) {
        if (t < 0 || t >= (1L << 30)) continue;
        ++checked;
        if (elbm::div_extent((int)t, rn) != t / n) ++bad;
      }
    }
  }
  const int big[] = {1 << 30, (1 << 30) - 1, 999983, 65535, 715827883};
  for (int n : big) {
    const double rn = 1.0 / n;
    for (long t = 0; t < (1L << 30); t += n / 5 + 7919) {
      const long u = (t / n + 1) * n - 1;
      ++checked;
      if (elbm::div_extent((int)t, rn) != t / n) ++bad;
      if (u < (1L << 30)) { ++checked; if (elbm::div_extent((int)u, rn) != u / n) ++bad; }
    }
  }
  std::printf("checked %ld mismatches %ld\n", checked, bad);
  return bad != 0;
}
