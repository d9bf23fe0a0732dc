// Shapes of the triangular solves' panels, shared by the host planner and
// the device kernels (no HIP types here: the planner is plain C++).
#pragma once

namespace condest {

// A block solves a panel with 64 row groups of 16 lanes: a panel of kPanel
// rows has one row per group, one of kMaxPanelRows two. The single-side
// solves use kMaxPanelRows-row panels, the several-sides solves kPanel-row
// ones.
constexpr int kPanel = 64;
constexpr int kMaxPanelRows = 128;
constexpr int kMaxSlicesDev = 64;  // most slices a heavy panel is cut into
// The tasks of a solve are dealt to kTaskLists lists, each handed out by its
// own ticket counter; the counters sit kTicketStride unsigned apart (one
// 128-byte line each), kSolveTickets unsigned per solve.
constexpr int kTaskLists = 8;
constexpr int kTicketStride = 32;
constexpr int kSolveTickets = kTaskLists * kTicketStride;

}  // namespace condest
