// Host-side check of the LDS staging tables the band builder makes for the extension and the
// fused sweep: for every workgroup, every LDS address that the kernels form for a node lies
// inside the workgroup's staged range and holds the band index that the gather form of the
// same pass reads.  Also checks the grouped patch rows of the learned smoother.  Prints one line per level and "ALL OK" or "FAIL"; exit status 1 on a
// mismatch.
#include <cstdio>
#include <string>
#include <vector>

#include "cpm_internal.h"

using namespace cpm;

static long check_level(const HostLevel& H, int dim) {
  const int S = dim == 2 ? 4 : 16, SX = dim == 2 ? 2 : 16, SR = S + SX;
  const int64_t n = H.n, nb = (n + kExtBlock - 1) / kExtBlock;
  const int32_t xmask = (1 << kXoffBits) - 1;
  long bad = 0;
  for (int64_t b = 0; b < nb; ++b) {
    const int32_t e0 = H.blkE[b], e1 = H.blkE[b + 1];
    for (int32_t e = e0; e < e1; ++e) bad += H.gidx[e] < 0 || H.gidx[e] >= n;
    const int32_t q0 = H.blkG[b] * S;
    for (int64_t k = b * kExtBlock; k < std::min<int64_t>(n, (b + 1) * kExtBlock); ++k) {
      const int32_t lg = H.packedL[k] >> kXoffBits, xo = H.packedL[k] & xmask;
      const int32_t gid = H.packed[k] >> kXoffBits, xg = H.packed[k] & xmask;
      bad += xo != xg;
      // extension: S runs of 4
      for (int s = 0; s < S; ++s)
        for (int a = 0; a < 4; ++a) {
          const int32_t L = H.lorg[q0 + lg * S + s] + xo + a, G = H.origin[(size_t)gid * S + s] + xg + a;
          bad += L < 0 || L >= e1 - e0 || H.gidx[e0 + L] != G;
        }
      if (H.blkE2.empty()) continue;
      // fused sweep: S runs of 6 (x0-1 .. x0+4), SX cross runs of 4
      const int32_t f0 = H.blkE2[b], f1 = H.blkE2[b + 1];
      const int32_t* org = &H.lorg2[(size_t)(H.blkG[b] + lg) * SR];
      for (int s = 0; s < S; ++s)
        for (int a = 0; a < 6; ++a) {
          const int32_t L = org[s] + xo - 1 + a, G = H.origin[(size_t)gid * S + s] + xg - 1 + a;
          bad += L < 0 || L >= f1 - f0 || H.gidx2[f0 + L] != G || G < 0 || G >= n;
        }
      for (int s = 0; s < SX; ++s)
        for (int a = 0; a < 4; ++a) {
          const int32_t L = org[S + s] + xo + a, G = H.originX[(size_t)gid * SX + s] + xg + a;
          bad += L < 0 || L >= f1 - f0 || H.gidx2[f0 + L] != G || G < 0 || G >= n;
        }
    }
  }
  return bad;
}

// Learned-smoother patch rows in grouped form: for every node and every row with a present
// node, the group's row plus the node's offset is the node's own row.
static long check_patches(const HostLevel& H, int dim) {
  if (!H.patchOK) return 0;
  const int rows = dim == 2 ? 3 : 9;
  const int64_t n = H.n, G = H.patchGroups;
  long bad = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t g = H.patchPk[i] >> kPatchBits;
    const int32_t t = H.patchPk[i] & (kPatchRun - 1);
    if (g < 0 || g >= G) {
      ++bad;
      continue;
    }
    for (int r = 0; r < rows; ++r)
      if ((H.patchMask[i] >> (3 * r)) & 7u) bad += H.patchBase[(size_t)(r * G + g)] + t != H.patchRow[(size_t)(r * n + i)];
  }
  return bad;
}

int main() {
  struct Case {
    cpm_surface s;
    double h;
    int levels, dim;
  };
  const Case cases[] = {
      {{CPM_CIRCLE, {0.0, 0.0, 0.0}, 1.0, 0.0}, 1.0 / 256, 5, 2},
      {{CPM_CIRCLE, {0.1, -0.05, 0.0}, 0.8, 0.0}, 1.0 / 64, 3, 2},
      {{CPM_SPHERE, {0.0, 0.0, 0.0}, 1.0, 0.0}, 1.0 / 32, 4, 3},
      {{CPM_SPHERE, {0.1, -0.2, 0.05}, 1.0, 0.0}, 1.0 / 24, 3, 3},
      {{CPM_TORUS, {0.0, 0.0, 0.0}, 1.0, 0.4}, 1.0 / 32, 3, 3},
      {{CPM_DZIUK, {0.0, 0.0, 0.0}, 1.0, 0.0}, 1.0 / 16, 2, 3},
  };
  long fails = 0;
  for (const Case& c : cases) {
    const cpm_grid g{c.h, c.levels, 0.0};
    std::vector<HostLevel> lv;
    std::string err;
    if (build_host_levels(c.s, g, c.dim, lv, err) != CPM_OK) {
      std::printf("build failed: %s\n", err.c_str());
      return 1;
    }
    for (size_t l = 0; l < lv.size(); ++l) {
      const long bad = check_level(lv[l], c.dim) + check_patches(lv[l], c.dim);
      std::printf("kind %d h = 1/%g level %zu: n = %ld, sweep tables %s, patch groups %ld, mismatches %ld\n",
                  c.s.kind, 1.0 / c.h, l, (long)lv[l].n, lv[l].blkE2.empty() ? "absent" : "present",
                  (long)lv[l].patchGroups, bad);
      fails += bad;
    }
  }
  std::printf(fails ? "FAIL\n" : "ALL OK\n");
  return fails ? 1 : 0;
}
