// Panel schedules of the sparse triangular solves (Algorithm 2's four
// solves with the LU factors): host planning and the device layout of one
// solve's arrays (plain C++; the upload is in panels_upload.hpp). Shared by
// the single-matrix plan and the batch.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "internal.hpp"
#include "solve_consts.hpp"

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
  kOffRp, kOffCol, kOffVal, kOffSplit, kPartials, kWinv, kWoff, kTaskRec, kTaskRp, kTaskSp,
  kSlotGroup, kTriSlots
};

// A strictly lower-triangular factor in solve order, cut into panels of at
// most prows consecutive rows, each split into the entries left of the panel
// and the entries inside it, plus the order in which panels are handed out.
struct PanelCsr {
  int32_t n = 0;
  int32_t prows = kPanel;  // most rows of a panel: 64 or 128 (kMaxPanelRows)
  std::vector<int64_t> off_rp, in_rp, off_split;
  std::vector<int32_t> off_col, in_col;
  std::vector<double> off_val, in_val;
  std::vector<int32_t> pstart;  // panel p holds rows [pstart[p], pstart[p+1])
  std::vector<int32_t> panel_split, panel_slot;  // slices per panel, first slot of a split panel
  std::vector<int32_t> task_panel, task_kind;    // tasks in dependency-level order
  std::vector<int32_t> task_level;               // dependency level of each task's panel
  std::vector<int32_t> task_group;  // joined schedules: the id of the block each task belongs to
  // Device order. Task k (in the order above) is dealt to list k mod
  // kTaskLists; list l is the slots [list_off[l], list_off[l+1]), its tasks
  // in dependency order, and task k sits at slot task_slot[k]. The arrays
  // below are indexed by slot.
  std::vector<int32_t> list_off, task_slot;
  // per slot: panel, kind, first row, rows, slices, first slot, and the
  // offset of its panel's inverse in winv as two 32-bit halves (low, high)
  std::vector<int32_t> task_rec;
  // per slot: the off-panel row pointers of its panel's rows (prows + 1
  // values, the last repeated past the panel's end) and their split points
  // (prows values, 0 past the end), so a block loads them together
  // with the record instead of after it
  std::vector<int64_t> task_rp, task_sp;
  // joined schedules, per slot: the block (a batch keeps each list's slots
  // of the blocks that still run)
  std::vector<int32_t> slot_group;
  // inverse of each panel's triangle, lower rows packed ((r, c) at
  // r (r + 1) / 2 + c); panel p's at winv[woff[p]]
  std::vector<double> winv;
  std::vector<int64_t> woff;
  int32_t levels = 0;
  int32_t nslots = 0;
};

// Panels, slices and tasks of a strictly lower factor t (rows in solve order).
PanelCsr split_panels(const HostCsr& t, int32_t prows);
// Schedules of independent diagonal blocks joined into one: parts[k] is the
// schedule of the block whose first row (in solve order) is offsets[k], the
// blocks in increasing offset order, contiguous. Panels, slots and inverses
// are concatenated; the tasks of all blocks are merged by dependency level
// (then block, then their own order), so the blocks' levels overlap; each
// task records groups[k] of its block.
PanelCsr merge_panels(const std::vector<const PanelCsr*>& parts, const std::vector<int64_t>& offsets,
                      const std::vector<int32_t>& groups);
// The inverse of every panel's triangle with diagonal diag (nullptr: unit);
// completes the task records (inverse offsets, row pointers).
void invert_panels(PanelCsr& s, const double* diag);
// Row i -> n-1-i and column j -> n-1-j: an upper factor becomes lower.
HostCsr reverse_order(const HostCsr& u);

// One solve on the host from the device-ready data, tasks in dependency
// order (in: right-hand side, gathered through `gather` when given); false
// when a task would read a value or slot that only a later task writes.
bool replay_solve(const PanelCsr& t, const int32_t* gather, const double* in, double* out);

// Workspace offsets of one solve's arrays for K right-hand sides (the slice
// partial slots hold K values per row).
void tri_layout(const PanelCsr& t, int K, Layout& L, size_t* off);

}  // namespace condest
