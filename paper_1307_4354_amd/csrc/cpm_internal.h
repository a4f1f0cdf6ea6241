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
  std::vector<int32_t> runE;   // 4^(dim-1) * n: first node of each x-run of the cubic stencil
  std::vector<int32_t> nbr;    // 2*dim * n: -x,+x,-y,+y,-z,+z neighbours, -1 if absent
  std::vector<double> fracP;   // dim * n: frac(cp / (2h)) (prolongation from level+1)
  std::vector<int32_t> runP;   // 2^(dim-1) * n: x-runs in level+1's band
  std::vector<double> fracR;   // dim * n: frac(cp / (h/2)) (restriction from level-1)
  std::vector<int32_t> runR;   // 2^(dim-1) * n: x-runs in level-1's band
};

// Device copies of one level's addressing.
struct DevLevel {
  int64_t n = 0;
  double h = 0.0;
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
};

// Build every level of the band hierarchy on the host.  Returns CPM_OK or an error with
// a message in `err`.
cpm_status build_host_levels(const cpm_surface& s, const cpm_grid& g, int dim,
                             std::vector<HostLevel>& levels, std::string& err);

void set_error(const std::string& msg);

}  // namespace cpm
