// Internal structures of libcpm shared by the host band builder, the kernels and the
// C ABI layer.  Not part of the public interface.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/cpm.h"

namespace cpm {

// Host-side band of one grid level (Sec. 3.1): nodes in x-fastest lexicographic order.
struct HostLevel {
  int dim = 0;
  double h = 0.0;
  double lam2 = 0.0;
  int64_t n = 0;
  int64_t lo[3] = {0, 0, 0};   // lower corner of the index box
  int64_t ext[3] = {1, 1, 1};  // extents of the index box
  std::vector<int32_t> idx;    // n * dim, row-major grid multi-indices
  std::vector<double> cp;      // n * dim, row-major closest points
  std::vector<int32_t> map;    // dense index box -> band index (-1 = not in band)
  // addressing, structure of arrays (slot-major: array[slot * n + i])
  std::vector<double> fracE;   // dim * n: frac(cp / h) for the cubic stencil
  std::vector<double> qdiag;   // n: (E N)_ii, so that diag(A) = delta - qdiag
  std::vector<double> q1diag;  // n: the same for Remark 3.2's operator (linear E in front of L)
  std::vector<int32_t> runE;   // 4^(dim-1) * n: first node of each x-run of the cubic stencil
  std::vector<int32_t> nbr;    // 2*dim * n: -x,+x,-y,+y,-z,+z neighbours, -1 if absent
  // extension in stencil order: nodes sorted by the base of their cubic stencil (z, y, x);
  // consecutive nodes with the same (y, z) base and the same row segments form a group
  // whose 4^(dim-1) x-run starts are stored once: run(s) = origin[gid][s] + xoff.
  std::vector<int32_t> perm;    // n: processing slot k -> band index
  std::vector<int32_t> packed;  // n: (gid << kXoffBits) | xoff
  std::vector<int32_t> packedB; // n: the same, indexed by band position
  std::vector<int32_t> origin;  // ngroups * 4^(dim-1)
  std::vector<double> fracK;    // dim * n: fractions in processing order
  int64_t ngroups = 0;
  // LDS staging of the extension: per workgroup of kExtBlock consecutive stencil slots, the
  // g values its stencils read (gidx, in LDS order) and, per local group, the LDS offset of
  // each x-run for xoff = 0 (lorg); packedL[k] = (local group << kXoffBits) | xoff
  std::vector<int32_t> blkE;    // nblocks + 1: prefix of staged values
  std::vector<int32_t> gidx;    // staged g indices
  std::vector<int32_t> blkG;    // nblocks + 1: prefix of local groups
  std::vector<int32_t> lorg;    // local groups * 4^(dim-1)
  std::vector<int32_t> packedL; // n
  int32_t maxE = 0, maxG = 0;   // largest staged set / local-group count of one workgroup
  int32_t extNpt = 1;           // workgroup of kExtBlock * extNpt stencil slots
  // Laplacian neighbours of interpolation-stencil nodes only (B_interp, ascending): the
  // +-x neighbours are j -+ 1, the others stored as -y,+y(,-z,+z) slot-major
  std::vector<int32_t> ilist;   // m
  std::vector<int32_t> nbrI;    // (2*dim-2) * m
  // the same list as segments of consecutive band entries whose +-y, +-z neighbours are
  // consecutive band entries too: per segment {first list position, first band index, the
  // 2*dim-2 neighbours of that node} (kNsumSegWords ints); per chunk of kNsumChunk list
  // positions the segment holding its first position, per position its segment's offset from
  // that one (< kNsumChunk, so one byte)
  std::vector<int32_t> nsSeg;
  std::vector<int32_t> nsChunkSeg;
  std::vector<uint8_t> nsSegOff;
  // the residual that the restriction into level+1 reads is needed only at the fine nodes of
  // its linear stencils (about a third of a level): the LDS-staged extension's tables over
  // those nodes alone, in this level's stencil order (their groups and run origins are the
  // level's own); empty on the coarsest level and when the level has no staging tables
  int64_t rsN = 0;
  std::vector<int32_t> rsPerm, rsPackedL, rsBlkE, rsGidx, rsBlkG, rsLorg;
  std::vector<double> rsFrac;  // dim * rsN, slot order
  int32_t rsMaxE = 0, rsMaxG = 0, rsNpt = 1;
  // fused sweep (E f + (E N) u in one pass): per stencil group, the band index of the first
  // node of each cross row of the stencil widened by the axis neighbours, for the group's
  // reference x (rows (y0-1, z0+c), (y0+4, z0+c), (y0+b, z0-1), (y0+b, z0+4) in 3-D; (y0-1),
  // (y0+4) in 2-D).  fusedOK is false when some node's cross rows do not follow that pattern.
  std::vector<int32_t> originX;
  bool fusedOK = false;
  // LDS staging of the fused sweep, on the extension's workgroups and local groups (blkG,
  // packedL): the u values the widened stencils read (gidx2) and, per local group, the LDS
  // offsets of its 4^(dim-1) rows (widened to 6 nodes) then of its cross rows (lorg2)
  std::vector<int32_t> blkE2;   // nblocks + 1: prefix of staged values
  std::vector<int32_t> gidx2;   // staged u indices
  std::vector<int32_t> lorg2;   // local groups * (4^(dim-1) + cross rows)
  int32_t maxE2 = 0;            // largest staged set of one workgroup
  // learned smoother (two finest levels): 3^dim grid patch of every node, in band order;
  // row (dy, dz) holds the band index of (x - 1, y + dy, z + dz) (virtual when that
  // node is absent), mask bit (dx+1) + 3 (dy+1) + 9 (dz+1) marks nodes that are present
  std::vector<int32_t> patchRow;  // 3^(dim-1) * n
  std::vector<uint32_t> patchMask;  // n
  bool patchOK = false;
  // the same rows stored once per group of consecutive nodes whose present rows all shift by
  // one band entry per node: patchBase[r * ngroups + g] + t is row r of the t-th node of
  // group g (t < kPatchRun); patchPk[i] = (group << kPatchBits) | t
  std::vector<int32_t> patchBase;
  std::vector<int32_t> patchPk;
  int64_t patchGroups = 0;
  // tiled sweep (3-D levels of at least kTileMinNodes nodes): nodes grouped by the tile of
  // kTileX x kTileY x kTileZ grid cells that holds their stencil base; one workgroup per tile
  // stages u (and f) over the tile's box, the stencils widened by the Laplacian's reach, in
  // LDS, forms f + N u there and interpolates it.  Per tile: slot range, box origin, and per
  // box row (y, z) the band index of its first in-band node and the presence mask of its
  // cells.  Per slot: band index, local coordinates, and the fractions in slot order.
  int64_t ntiles = 0;
  std::vector<int32_t> tileSlot;  // ntiles + 1
  std::vector<int32_t> tileOrg;   // 3 * ntiles: box origin (x, y, z)
  std::vector<int32_t> tileRow;   // 2 * kBoxRows * ntiles: {first band index, cell mask}
  std::vector<int32_t> tperm;     // n: slot -> band index
  std::vector<int32_t> tloc;      // n: local base (5 bits per axis), own box cell, in-box flag
  std::vector<double> fracT;      // 3 * n: fractions in slot order
  std::vector<double> fracP;   // dim * n: frac(cp / (2h)) (prolongation from level+1)
  // cubic interpolation from level+1 at this level's closest points (4^(d-1) runs of 4, and
  // the fractions), the nested-iteration step of the full-multigrid start; empty when some
  // stencil leaves the coarse band
  std::vector<int32_t> runP3;
  std::vector<double> fracP3;
  std::vector<int32_t> runP;   // 2^(dim-1) * n: x-runs in level+1's band
  std::vector<double> fracR;   // dim * n: frac(cp / (h/2)) (restriction from level-1)
  std::vector<int32_t> runR;   // 2^(dim-1) * n: x-runs in level-1's band
};

constexpr int kXoffBits = 6;  // x-offset bits of a stencil group: a group lies inside one Morton
                              // block (offsets below 8), or, in the plain order, is cut at 64
                              // nodes; the group id keeps 25 bits (levels of 10^8 nodes)
constexpr int kPatchBits = 8;  // node offset bits of a learned-smoother patch group
constexpr int kPatchRun = 1 << kPatchBits;
constexpr int kExtBlock = 256;      // workgroup size of the LDS-staged extension
constexpr int64_t kExtNptMinNodes = 4 << 20;  // levels at least this large (without the fused
                                              // sweep's tables) stage for 2 slots per thread
constexpr int kMaxStaged = 8192;    // staged values per workgroup above which a level keeps the gather path
constexpr int kNsumChunkBits = 8;  // neighbour-sum segment tables: chunks of 256 list positions
constexpr int kNsumChunk = 1 << kNsumChunkBits;
constexpr int kNsumSegWords = 6;   // per segment: first position, first band index, 4 neighbours
constexpr int kMaxDynLds = 65536;  // dynamic LDS bytes a staged extension workgroup may take
constexpr int kMaxGroups = 1 << (31 - kXoffBits);
// largest level that gets the fused-sweep addressing
constexpr int64_t kFusedMaxNodes = 2 << 20;
// levels up to this size sweep with the fused pass unless the autotuner decides otherwise
constexpr int64_t kFusedDefaultNodes = 128 << 10;

// tiled sweep geometry: tile of kTileX x kTileY x kTileZ stencil bases; its box spans the
// stencils (+3) widened by one cell on each side (the Laplacian of the stencil nodes)
constexpr int kTileX = 8, kTileY = 8, kTileZ = 8;
constexpr int kBoxX = kTileX + 5, kBoxY = kTileY + 5, kBoxZ = kTileZ + 5;
constexpr int kBoxRows = kBoxY * kBoxZ;
constexpr int kBoxCells = kBoxX * kBoxRows;
constexpr int kGX = kBoxX - 2, kGY = kBoxY - 2, kGZ = kBoxZ - 2;  // the stencils' box
constexpr int kGCells = kGX * kGY * kGZ;
constexpr int64_t kTileMinNodes = 1 << 18;
constexpr int kTileBlock = 256;

// Device copies of one level's addressing.
struct DevLevel {
  int64_t n = 0;
  int64_t m = 0;        // |B_interp|
  int64_t ngroups = 0;
  double h = 0.0;
  bool band_order = false;  // extension visits nodes in band order (packedB, fracE)
  bool lds = false;         // LDS-staged extension tables present
  bool use_lds = false;     // extension runs LDS-staged (else gathers through L1)
  int ext_block = 256;      // workgroup size of the gather extension
  bool ext_prefetch = false;  // LDS-staged extension loads the node's own data before staging
  bool prefetch_forced = false;  // set by CPM_EXT_PREFETCH
  int nsum_block = 256;     // workgroup size of the neighbour sum and transfers
  int sweep_block = 256;    // workgroup size of the fused sweep
  bool sweep_forced = false;  // fused / split chosen by the CPM_SWEEP environment variable
  int32_t maxE = 0, maxG = 0;
  int ext_npt = 1;
  int32_t* blkE = nullptr;
  int32_t* gidx = nullptr;
  int32_t* blkG = nullptr;
  int32_t* lorg = nullptr;
  int32_t* packedL = nullptr;
  int32_t* perm = nullptr;
  int32_t* packed = nullptr;
  int32_t* packedB = nullptr;
  int32_t* origin = nullptr;
  double* fracK = nullptr;
  float* fracK32 = nullptr;
  int32_t* ilist = nullptr;
  int32_t* nbrI = nullptr;
  int32_t* nsSeg = nullptr;
  int32_t* nsChunkSeg = nullptr;
  uint8_t* nsSegOff = nullptr;
  int64_t rs_n = 0;  // residual-for-restriction subset (see HostLevel::rsN); 0: full level
  int32_t *rs_perm = nullptr, *rs_packedL = nullptr, *rs_blkE = nullptr, *rs_gidx = nullptr, *rs_blkG = nullptr,
          *rs_lorg = nullptr;
  double* rs_frac = nullptr;
  float* rs_frac32 = nullptr;
  int32_t rs_maxE = 0, rs_maxG = 0, rs_npt = 1;
  int32_t* runE = nullptr;
  int32_t* nbr = nullptr;
  double* fracE = nullptr;
  float* fracE32 = nullptr;
  int32_t* runP = nullptr;
  double* fracP = nullptr;
  float* fracP32 = nullptr;
  int32_t* runR = nullptr;
  double* fracR = nullptr;
  float* fracR32 = nullptr;
  int32_t* originX = nullptr;
  bool sweep_lds = false;      // LDS staging tables of the fused sweep present
  bool use_sweep_lds = false;  // fused sweep runs LDS-staged (else gathers through L1)
  int32_t maxE2 = 0;
  int32_t* blkE2 = nullptr;
  int32_t* gidx2 = nullptr;
  int32_t* lorg2 = nullptr;
  int32_t* runP3 = nullptr;  // full-multigrid interpolation from level+1 (cubic)
  double* fracP3 = nullptr;
  double* qdiag = nullptr;  // (E N)_ii
  double* q1diag = nullptr; // delta - diag(A) of Remark 3.2's operator
  double* wd1 = nullptr;    // omega / diag(A) of that operator (set per c, omega)
  double* acoef = nullptr;  // variable diffusion coefficient a(cp(x_i)) (cpm_set_diffusion)
  double* vcD = nullptr;    // c + sigma_i of the flux-form operator, for vc_c
  double* wd = nullptr;     // omega / diag(A) of the standard relaxation (set per c, omega)
  uint8_t* parity = nullptr;  // colour of the red-black sweeps: parity of the grid index sum
  double* wdR = nullptr;      // wd on red nodes, 0 on black ones
  double* wdB = nullptr;      // wd on black nodes, 0 on red ones
  bool fusedOK = false;
  bool fused = false;  // sweeps as one fused pass instead of neighbour sum + extension
  int32_t* patchRow = nullptr;   // grouped rows (HostLevel::patchBase), rows x patchGroups
  int32_t* patchPk = nullptr;    // per node (group << kPatchBits) | offset
  int64_t patchGroups = 0;
  uint32_t* patchMask = nullptr;
  // tiled sweep (HostLevel::tileSlot ...); use_tile: the level sweeps with it
  int64_t ntiles = 0;
  bool use_tile = false;
  int32_t* tileSlot = nullptr;
  int32_t* tileOrg = nullptr;
  int32_t* tileRow = nullptr;
  int32_t* tperm = nullptr;
  int32_t* tloc = nullptr;
  double* fracT = nullptr;
  float* fracT32 = nullptr;
};

// Build every level of the band hierarchy on the host.  Returns CPM_OK or an error with
// a message in `err`.
cpm_status build_host_levels(const cpm_surface& s, const cpm_grid& g, int dim,
                             std::vector<HostLevel>& levels, std::string& err);

void set_error(const std::string& msg);

// Reach of an analytic surface (level sets: a curvature bound).
double surface_reach(const cpm_surface& s);

// OpenMP threads of the calling host thread's band construction.
void set_host_build_threads(int n);

}  // namespace cpm
