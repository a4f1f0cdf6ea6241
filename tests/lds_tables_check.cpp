// Host-side check of the LDS staging tables the band builder makes for the extension and the
// fused sweep: for every workgroup, every LDS address that the kernels form for a node lies
// inside the workgroup's staged range and holds the band index that the gather form of the
// same pass reads.  Also checks the grouped patch rows of the learned smoother.  Prints one line per level and "ALL OK" or "FAIL"; exit status 1 on a
// mismatch.
#include <algorithm>
#include <cstdlib>
#include <array>
#include <cstdio>
#include <string>
#include <vector>

#include "cpm_internal.h"

using namespace cpm;

static long check_level(const HostLevel& H, int dim) {
  const int S = dim == 2 ? 4 : 16, SX = dim == 2 ? 2 : 16, SR = S + SX;
  const int64_t wg = (int64_t)kExtBlock * H.extNpt;
  const int64_t n = H.n, nb = (n + wg - 1) / wg;
  const int32_t xmask = (1 << kXoffBits) - 1;
  long bad = 0;
  if (H.extNpt != 1 && !H.blkE2.empty()) ++bad;  // the fused sweep runs one slot per thread
  for (int64_t b = 0; b < nb; ++b) {
    const int32_t e0 = H.blkE[b], e1 = H.blkE[b + 1];
    for (int32_t e = e0; e < e1; ++e) bad += H.gidx[e] < 0 || H.gidx[e] >= n;
    const int32_t q0 = H.blkG[b] * S;
    for (int64_t k = b * wg; k < std::min<int64_t>(n, (b + 1) * wg); ++k) {
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

// Learned-smoother patch rows in grouped form: for every node and every present node of its
// 3^dim patch, the address the kernels form (the group's row plus the node's offset plus dx,
// one less for the +1 node of a row whose middle node is absent) is the band index of that
// grid node, found here by a binary search of the sorted grid keys.  Counts the gapped rows.
static long check_patches(const HostLevel& H, int dim, long* gaps) {
  if (!H.patchOK) return 0;
  const int rows = dim == 2 ? 3 : 9;
  const int64_t n = H.n, G = H.patchGroups;
  std::vector<std::array<int32_t, 3>> keys((size_t)n);
  for (int64_t i = 0; i < n; ++i)
    keys[(size_t)i] = {dim == 3 ? H.idx[(size_t)(i * dim + 2)] : 0, H.idx[(size_t)(i * dim + 1)],
                       H.idx[(size_t)(i * dim)]};
  auto find = [&](int32_t x, int32_t y, int32_t z) -> int64_t {
    const std::array<int32_t, 3> k = {z, y, x};
    auto it = std::lower_bound(keys.begin(), keys.end(), k);
    return (it != keys.end() && *it == k) ? (int64_t)(it - keys.begin()) : -1;
  };
  long bad = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t g = H.patchPk[i] >> kPatchBits;
    const int32_t t = H.patchPk[i] & (kPatchRun - 1);
    if (g < 0 || g >= G) {
      ++bad;
      continue;
    }
    const int32_t* m = &H.idx[(size_t)(i * dim)];
    for (int r = 0; r < rows; ++r) {
      const uint32_t rm = (H.patchMask[i] >> (3 * r)) & 7u;
      const int dy = r % 3 - 1, dz = dim == 3 ? r / 3 - 1 : 0;
      const int gap = rm == 5u;
      *gaps += gap;
      for (int dx = 0; dx < 3; ++dx) {
        const int64_t j = find(m[0] + dx - 1, m[1] + dy, dim == 3 ? m[2] + dz : 0);
        const bool present = (rm >> dx) & 1u;
        if (present != (j >= 0)) {
          ++bad;
          continue;
        }
        if (!present) continue;
        const int64_t addr = (int64_t)H.patchBase[(size_t)(r * G + g)] + t + dx - (dx == 2 ? gap : 0);
        bad += addr != j;
      }
    }
  }
  return bad;
}

// Tiled-sweep tables: every tile's slots are its nodes; for every node, every stencil node
// (and each of its six Laplacian neighbours) lies in its box row's staged x range, at the
// band index the gather form of the extension reads; the node's own box cell, when flagged,
// holds the node itself.  Returns mismatches; *tiles gets the tile count.
static long check_tiles(const HostLevel& H, long* tiles) {
  *tiles = H.ntiles;
  if (H.ntiles <= 0) return 0;
  const int64_t n = H.n;
  long bad = 0;
  std::vector<int> seen((size_t)n, 0);
  auto row_index = [&](int64_t t, int y, int z, int x, int64_t* idx) -> bool {
    if (y < 0 || y >= kBoxY || z < 0 || z >= kBoxZ || x < 0 || x >= kBoxX) return false;
    const int32_t* rr = &H.tileRow[(size_t)(2 * (t * kBoxRows + z * kBoxY + y))];
    const uint32_t mask = (uint32_t)rr[1];
    if (!((mask >> x) & 1u)) return false;
    *idx = (int64_t)rr[0] + __builtin_popcount(mask & ((1u << x) - 1u));
    return *idx >= 0 && *idx < n;
  };
  for (int64_t t = 0; t < H.ntiles; ++t) {
    const int64_t s0 = H.tileSlot[(size_t)t], s1 = H.tileSlot[(size_t)t + 1];
    if (s1 < s0) ++bad;
    for (int64_t k = s0; k < s1; ++k) {
      const int32_t i = H.tperm[(size_t)k];
      if (i < 0 || i >= n) {
        ++bad;
        continue;
      }
      seen[(size_t)i]++;
      const int32_t loc = H.tloc[(size_t)k];
      const int lx = loc & 31, ly = loc >> 5 & 31, lz = loc >> 10 & 31;
      if (lx >= kTileX || ly >= kTileY || lz >= kTileZ) ++bad;
      for (int c = 0; c < 4; ++c)
        for (int b = 0; b < 4; ++b)
          for (int a = 0; a < 4; ++a) {
            const int x = lx + a + 1, y = ly + b + 1, z = lz + c + 1;  // box cell of the stencil node
            int64_t j = -1;
            if (!row_index(t, y, z, x, &j) || j != (int64_t)H.runE[(size_t)((b + 4 * c) * n + i)] + a) {
              ++bad;
              continue;
            }
            const int d[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
            for (int q = 0; q < 6; ++q) {
              int64_t jn = -1;
              if (!row_index(t, y + d[q][1], z + d[q][2], x + d[q][0], &jn) ||
                  jn != (int64_t)H.nbr[(size_t)(q * n + j)])
                ++bad;
            }
          }
      for (int a = 0; a < 3; ++a)
        bad += H.fracT[(size_t)(a * n + k)] != H.fracE[(size_t)(a * n + i)];
      if (loc >> 30 & 1) {
        int64_t j = -1;
        if (!row_index(t, loc >> 20 & 31, loc >> 25 & 31, loc >> 15 & 31, &j) || j != i) ++bad;
      }
    }
  }
  for (int64_t i = 0; i < n; ++i) bad += seen[(size_t)i] != 1;
  return bad;
}

// Neighbour-sum segment tables: every list position's band index and +-y, +-z neighbours, as
// the segmented kernel forms them, equal the per-node lists.
static long check_nsum_segments(const HostLevel& H, int dim, long* nseg) {
  const int64_t m = (int64_t)H.ilist.size();
  const int nq = 2 * dim - 2;
  *nseg = (long)(H.nsSeg.size() / kNsumSegWords);
  if ((int64_t)H.nsSegOff.size() != m || (int64_t)H.nsChunkSeg.size() != (m + kNsumChunk - 1) / kNsumChunk) return 1;
  long bad = 0;
  for (int64_t k = 0; k < m; ++k) {
    const int64_t sidx = (int64_t)H.nsChunkSeg[(size_t)(k >> kNsumChunkBits)] + H.nsSegOff[(size_t)k];
    if (sidx < 0 || sidx >= *nseg) {
      ++bad;
      continue;
    }
    const int32_t* sg = &H.nsSeg[(size_t)(sidx * kNsumSegWords)];
    const int32_t t = (int32_t)k - sg[0];
    bad += t < 0 || sg[1] + t != H.ilist[(size_t)k];
    for (int q = 0; q < nq; ++q) bad += sg[2 + q] + t != H.nbrI[(size_t)(q * m + k)];
  }
  return bad;
}

// Residual-for-restriction subset of level F (coarse level C): its slots are exactly the fine
// nodes C's restriction stencils read, in F's stencil order, and every LDS address its staged
// extension forms holds the band index the gather form reads for that node.
static long check_resid_subset(const HostLevel& F, const HostLevel* C, int dim, long* nsub) {
  *nsub = (long)F.rsN;
  if (!C) return F.rsN != 0;
  if (F.rsN == 0) return std::getenv("CPM_RESID_SUBSET") ? 0 : 1;
  const int S = dim == 2 ? 4 : 16, nr = 1 << (dim - 1);
  const int64_t n = F.n, nc = C->n, ns = F.rsN;
  const int32_t xmask = (1 << kXoffBits) - 1;
  long bad = 0;
  std::vector<char> need((size_t)n, 0), seen((size_t)n, 0);
  for (int r = 0; r < nr; ++r)
    for (int64_t j = 0; j < nc; ++j) {
      need[(size_t)C->runR[(size_t)(r * nc + j)]] = 1;
      need[(size_t)C->runR[(size_t)(r * nc + j)] + 1] = 1;
    }
  // the subset is the needed set, in increasing stencil-slot order
  std::vector<int64_t> slot_of((size_t)n, -1);
  for (int64_t k = 0; k < n; ++k) slot_of[(size_t)F.perm[(size_t)k]] = k;
  int64_t prev = -1;
  for (int64_t k = 0; k < ns; ++k) {
    const int32_t i = F.rsPerm[(size_t)k];
    bad += i < 0 || i >= n || !need[(size_t)i] || seen[(size_t)i] || slot_of[(size_t)i] <= prev;
    if (i >= 0 && i < n) {
      seen[(size_t)i] = 1;
      prev = slot_of[(size_t)i];
    }
  }
  for (int64_t i = 0; i < n; ++i) bad += need[(size_t)i] && !seen[(size_t)i];
  const int64_t wg = (int64_t)kExtBlock * F.rsNpt, nb = (ns + wg - 1) / wg;
  for (int64_t b = 0; b < nb; ++b) {
    const int32_t e0 = F.rsBlkE[(size_t)b], e1 = F.rsBlkE[(size_t)b + 1], q0 = F.rsBlkG[(size_t)b] * S;
    for (int64_t k = b * wg; k < std::min<int64_t>(ns, (b + 1) * wg); ++k) {
      const int32_t i = F.rsPerm[(size_t)k];
      const int32_t lg = F.rsPackedL[(size_t)k] >> kXoffBits, xo = F.rsPackedL[(size_t)k] & xmask;
      const int32_t gid = F.packedB[(size_t)i] >> kXoffBits, xg = F.packedB[(size_t)i] & xmask;
      bad += xo != xg;
      for (int s = 0; s < S; ++s)
        for (int a = 0; a < 4; ++a) {
          const int32_t L = F.rsLorg[(size_t)(q0 + lg * S + s)] + xo + a, G = F.origin[(size_t)gid * S + s] + xg + a;
          bad += L < 0 || L >= e1 - e0 || F.rsGidx[(size_t)(e0 + L)] != G;
        }
      for (int a = 0; a < dim; ++a) bad += F.rsFrac[(size_t)(a * ns + k)] != F.fracE[(size_t)(a * n + i)];
    }
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
      {{CPM_TORUS, {0.0, 0.0, 0.0}, 1.0, 0.25}, 1.0 / 16, 3, 3},  // gapped patch rows on level 1
      {{CPM_SPHERE, {0.0, 0.0, 0.0}, 1.0, 0.0}, 1.0 / 64, 2, 3},   // tiled-sweep tables on level 0
      {{CPM_TORUS, {0.05, 0.0, 0.0}, 1.0, 0.4}, 1.0 / 64, 2, 3},
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
      long gaps = 0, tiles = 0, nseg = 0, nsub = 0;
      const long bad = check_level(lv[l], c.dim) + check_patches(lv[l], c.dim, &gaps) + check_tiles(lv[l], &tiles) +
                       check_nsum_segments(lv[l], c.dim, &nseg) +
                       check_resid_subset(lv[l], l + 1 < lv.size() ? &lv[l + 1] : nullptr, c.dim, &nsub);
      std::printf("kind %d h = 1/%g level %zu: n = %ld, slots per thread %d, sweep tables %s, patch groups %ld, "
                  "gapped rows %ld, tiles %ld, sum segments %ld (%.1f nodes each), restriction subset %ld, mismatches %ld\n",
                  c.s.kind, 1.0 / c.h, l, (long)lv[l].n, (int)lv[l].extNpt, lv[l].blkE2.empty() ? "absent" : "present",
                  (long)lv[l].patchGroups, gaps, tiles, nseg, nseg ? (double)lv[l].ilist.size() / nseg : 0.0, nsub, bad);
      fails += bad;
    }
  }
  std::printf(fails ? "FAIL\n" : "ALL OK\n");
  return fails ? 1 : 0;
}
