// Helper launchers used by the host orchestration (enqueue only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gm {

hipError_t fill_i32(int32_t *p, int64_t count, int32_t v, hipStream_t s);
hipError_t iota_i32(int32_t *p, int64_t count, hipStream_t s);
hipError_t iota_i64(int64_t *p, int64_t count, int64_t start, hipStream_t s);
// Every vertex a source: usrc, slot_of and slot_row the identity on [0, n),
// info[0..8) cleared, in one launch.
hipError_t all_sources_setup(int32_t n, int32_t *usrc, int32_t *slot_of, int64_t *slot_row, int32_t *info,
                             hipStream_t s);
// slot_of[usrc[i]] = i
hipError_t scatter_slots(const int32_t *usrc, int32_t count, int32_t *slot_of, hipStream_t s);
// Listed sources src[rows] -> sorted unique sources on the device:
// first[v] = first row naming v (INT32_MAX if none), usrc[slot] (ascending),
// slot_row[slot] = first row, slot_of[v] (-1 if not a source), and, when
// count and mult are not NULL, mult[slot] = times listed; info[0] gets bit 1
// for an id outside [0, n), info[3] the number of unique sources.  marks,
// pos (n + 1) and scan_tmp (exclusive_scan_scratch_bytes(n)) are scratch.
hipError_t prepare_sources(const int32_t *src, int64_t rows, int32_t n, int32_t *first, int32_t *count,
                           int32_t *marks, int32_t *pos, void *scan_tmp, int32_t *usrc, int64_t *slot_row,
                           int32_t *slot_of, int32_t *mult, int32_t *info, hipStream_t s);
// The same for at most 4,096 rows on at most 131,072 vertices in two launches
// (a per-vertex pass that also lists the heavy vertices of the level kernel
// as launch_heavy_list does, then one workgroup ranking the listed vertices
// with a bit set in LDS); info[1] must be zero.  With host_info (pinned host
// memory, 8 ints; rows > 0) the ranking kernel also stores the final
// info[0..7] there, read once the stream has finished.
bool sources_ranked_small(int64_t rows, int32_t n);
hipError_t prepare_sources_small(const int32_t *src, int64_t rows, int32_t n, const int32_t *row_ptr,
                                 int32_t heavy_forced, int32_t *heavy, int32_t *first, int32_t *count,
                                 int32_t *usrc, int64_t *slot_row, int32_t *slot_of, int32_t *mult, int32_t *info,
                                 hipStream_t s, int32_t *host_info = nullptr);
// Rows r with first[src[r]] != r copy row first[src[r]] of ids/hops (k wide)
// and of the hop matrix (n wide, when not NULL).
hipError_t copy_dup_rows(const int32_t *src, int64_t rows, const int32_t *first, int32_t k, int32_t n, int32_t *ids,
                         uint8_t *hops, uint8_t *hop_matrix, hipStream_t s);
// bit 32 in *err unless every row is strictly increasing without self-loops
hipError_t check_sorted(int32_t n, const int32_t *rp, const int32_t *col, int *err, hipStream_t s);
// bits 128/256 in *err for malformed row pointers / ids of a packed batch whose
// offsets are already known to be monotone and consistent with the totals
hipError_t validate_batch(int32_t n_graphs, const int64_t *voff, const int64_t *eoff, const int32_t *rp,
                          const int32_t *col, int64_t total_v, int64_t total_e, int *err, hipStream_t s);
// packed per-graph CSR -> one CSR of the disjoint union (global ids)
hipError_t batch_to_union(int32_t n_graphs, const int64_t *voff, const int64_t *eoff, const int32_t *rp,
                          const int32_t *col, int64_t total_v, int64_t total_e, int32_t *urp,
                          int32_t *ucol, hipStream_t s);
// union CSR -> packed per-graph CSR with new edge offsets
hipError_t union_to_batch(int32_t n_graphs, const int64_t *voff, const int32_t *urp, const int32_t *ucol,
                          int64_t total_v, int64_t total_e_canon, int64_t *eoff_out, int32_t *rp_out,
                          int32_t *col_out, hipStream_t s);

}  // namespace gm
