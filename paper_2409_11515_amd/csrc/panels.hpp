// Panel schedules of the sparse triangular solves (Algorithm 2's four
// solves with the LU factors): host planning, the device layout of one
// solve's arrays, and their upload. Shared by the single-matrix plan and the
// batch.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"

namespace condest {

constexpr size_t kAlign = 256;

struct Layout {
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t o = (off + kAlign - 1) / kAlign * kAlign;
    off = o + bytes;
    return o;
  }
};

// Device arrays of one solve's panel structure (offsets into the workspace).
enum TriSlot {
  kOffRp, kOffCol, kOffVal, kOffSplit, kInRp, kInSplit, kInCol, kInVal,
  kPartials, kWinv, kWoff, kTaskRec, kTriSlots
};

// A strictly lower-triangular factor in solve order, cut into panels of at
// most kPanelRows consecutive rows, each split into the entries left of the
// panel and the entries inside it, plus the order in which panels are handed
// out. A row's in-panel entries list those on earlier 64-row sub-panels of
// its panel first; in_split marks where the entries of its own sub-panel start.
struct PanelCsr {
  int32_t n = 0;
  std::vector<int64_t> off_rp, in_rp, in_split, off_split;
  std::vector<int32_t> off_col, in_col;
  std::vector<double> off_val, in_val;
  std::vector<int32_t> pstart;  // panel p holds rows [pstart[p], pstart[p+1])
  std::vector<int32_t> panel_split, panel_slot;  // slices per panel, first slot of a split panel
  std::vector<int32_t> task_panel, task_kind;    // tasks in dependency-level order
  std::vector<int32_t> task_level;               // dependency level of each task's panel
  std::vector<int32_t> task_rec;  // per task: panel, kind, first row, rows, slices, slot, 0, 0
  // inverse of each sub-panel's triangle, lower rows packed; panel p's
  // sub-panel j at winv[woff[p] + j * kTriPacked]
  std::vector<double> winv;
  std::vector<int64_t> woff;
  int32_t levels = 0;
  int32_t nslots = 0;
};

// Panels, slices and tasks of a strictly lower factor t (rows in solve order).
PanelCsr split_panels(const HostCsr& t);
// Schedules of independent diagonal blocks joined into one: parts[k] is the
// schedule of the block whose first row (in solve order) is offsets[k], the
// blocks in increasing offset order, contiguous. Panels, slots and inverses
// are concatenated; the tasks of all blocks are merged by dependency level
// (then block, then their own order), so the blocks' levels overlap.
PanelCsr merge_panels(const std::vector<const PanelCsr*>& parts, const std::vector<int64_t>& offsets);
// The inverse of every sub-panel's triangle with diagonal diag (nullptr: unit).
void invert_panels(PanelCsr& s, const double* diag);
// Row i -> n-1-i and column j -> n-1-j: an upper factor becomes lower.
HostCsr reverse_order(const HostCsr& u);

// One solve on the host from the device-ready data, tasks in ticket order
// (in: right-hand side, gathered through `gather` when given); false when a
// task would read a value or slot that only a later ticket writes.
bool replay_solve(const PanelCsr& t, const int32_t* gather, const double* in, double* out);

// Workspace offsets of one solve's arrays for K right-hand sides (the slice
// partial slots hold K values per row).
void tri_layout(const PanelCsr& t, int K, Layout& L, size_t* off);
// Uploads them on `s` at ws + off[...], arms the partial slots, fills `out`.
int tri_upload(char* ws, const size_t* off, const PanelCsr& t, int K, hipStream_t s, DevTri& out);

}  // namespace condest
