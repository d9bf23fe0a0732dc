// Shapes of the triangular solves' panels, shared by the host planner and
// the device kernels (no HIP types here: the planner is plain C++).
#pragma once

namespace condest {

constexpr int kPanel = 64;         // rows of a sub-panel: one wave solves its triangle
constexpr int kMaxSlicesDev = 64;  // most slices a heavy panel is cut into
constexpr int kPanelRows = 64;     // rows of a panel: its sub-panels are solved in order by one block
constexpr int kTriPacked = kPanel * (kPanel + 1) / 2;  // entries of a packed 64-row triangle
// The tasks of a solve are dealt to kTaskLists lists, each handed out by its
// own ticket counter; the counters sit kTicketStride unsigned apart (one
// 128-byte line each), kSolveTickets unsigned per solve.
constexpr int kTaskLists = 8;
constexpr int kTicketStride = 32;
constexpr int kSolveTickets = kTaskLists * kTicketStride;

}  // namespace condest
