// Internal launchers of the gfx950 kernels (host side).  Every launcher
// enqueues on `stream` and returns the launch status; none synchronises.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace gm {

// ----------------------------------------------------------------- CSR ---
// Structural check of an input CSR.  Sets bits in *err (device int):
//   1 row_ptr[0] != 0, 2 row_ptr not monotone or outside [0, nnz],
//   4 row_ptr[n] != nnz, 8 col_idx entry outside [0, n).
hipError_t launch_validate_structure(int32_t n, int32_t nnz, const int32_t *row_ptr,
                                     const int32_t *col_idx, int *err, hipStream_t s);
// Symmetry check of a canonical CSR: bit 16 in *err if some (u, w) lacks (w, u).
hipError_t launch_check_symmetric(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                                  int *err, hipStream_t s);

// Scratch needed by launch_canonicalize for a graph of this size (bytes).
size_t canon_scratch_bytes(int32_t n, int32_t nnz);
// Canonical CSR (rows sorted, unique, no self-loops) of an arbitrary one.
// out_row_ptr: n + 1 entries; out_col: nnz entries (capacity).  The number of
// kept entries ends up in out_row_ptr[n], and also in *host_total when that
// is given (pinned host memory the kernel stores into; read it once the
// stream has finished; n > 0).
hipError_t launch_canonicalize(int32_t n, int32_t nnz, const int32_t *row_ptr,
                               const int32_t *col_idx, int32_t *out_row_ptr, int32_t *out_col,
                               void *scratch, hipStream_t s, int32_t *host_total = nullptr);

// Exclusive prefix sum of int32 `in` (len values) into `out` (len + 1 values,
// out[len] = total).  scratch: exclusive_scan_scratch_bytes(len).
size_t exclusive_scan_scratch_bytes(int64_t len);
hipError_t launch_exclusive_scan(const int32_t *in, int32_t *out, int64_t len, void *scratch,
                                 hipStream_t s);

// Stable LSD radix sort of (key, value) pairs by key bits [begin_bit,
// end_bit), 8 bits per pass, count < 2^31 (hipErrorInvalidValue otherwise).
// The passes alternate between (keys, vals) and (keys_alt, vals_alt); the
// result is in the _alt pair when *in_alt is set on return.  scratch:
// radix_sort_scratch_bytes(count).
size_t radix_sort_scratch_bytes(int64_t count);
template <typename K>
hipError_t radix_sort_pairs(K *keys, K *keys_alt, uint32_t *vals, uint32_t *vals_alt, int64_t count, int begin_bit,
                            int end_bit, void *scratch, hipStream_t s, bool *in_alt);

// ------------------------------------------------------ all-source BFS ---
// Multi-source bit-parallel BFS over groups of W = 64 * words sources.
// Layout of every state array: [group][vertex][word] of uint64.
struct MsbfsArgs {
    int32_t n;
    const int32_t *row_ptr;   // canonical CSR
    const int32_t *col;
    int32_t words;            // 64-bit words per vertex per group (1, 2, 4 or 8)
    int32_t groups;           // groups in this round
    int32_t slot0;            // first global slot of this round
    int32_t n_slots;          // slots in this round (<= groups * 64 * words)
    const int32_t *usrc;      // sorted unique sources, indexed by global slot
    int32_t n_usrc;           // total slots
    const int32_t *slot_of;   // vertex -> global slot or -1
    uint64_t *front[2];       // plane mode: rotating frontier / next arrays
    uint64_t *visited;
    uint64_t *planes;         // 8 bit-planes of the discovery level, plane-major
    size_t plane_stride;      // uint64 elements per plane (= groups * n * words)
    // History mode (hist_levels = H > 0): the frontier found at hop h is kept
    // in hist slot h - 1 for h <= H + 1 (two rotating slots H + 1, H + 2
    // beyond), so hops 1..H need no bit-plane commits: the transposes read
    // them from the history (up to each group's depth, found from the level
    // counters of the levels_run levels launched so far); only hops above H
    // go to the planes.  hist_levels = 0: plane mode (front[2] rotate).
    uint64_t *hist;
    int32_t hist_levels;
    int32_t levels_run;
    unsigned long long *stats; // [level][group][spread][field] counters of each level
    int32_t stats_groups;     // groups per stats level
    const int32_t *heavy;     // vertices of degree above heavy_deg
    int32_t n_heavy;
    int32_t heavy_deg;
    int32_t heavy_maxdeg;     // largest degree among them
    int32_t xcd_map;          // keep each group on one XCD when groups % 8 == 0
    int32_t hops_variant;     // hop-row writer: tiles per step / store kind (tuning)
    int32_t level_verts;      // (vertex, word) items per thread of the level kernel: 1, 2, 4 or 8
    const int32_t *planes_dev; // if not NULL: the transpose reads its plane count here (device)
    // Direction: levels 2..push_levels may run top-down (msbfs_push_kernel),
    // per group, when the frontier's edge-words * push_ratio < nnz * words;
    // the first fill then clears their next-frontier arrays.  0: bottom-up only.
    int32_t push_levels;
    int32_t push_ratio;
    int32_t nnz;
};
// Layout of the level counters: stats[((level * groups + g) * spread + slot) * fields + field]
// with fields {new bits, frontier words gathered (pull) or pushed (push),
// adjacency entries read, frontier words committed, edge-words of the items
// found}; a level's value is the sum over the spread slots.
int msbfs_stat_fields();
int msbfs_stat_spread();
// heavy[0 .. info[1]) = vertices of degree above the threshold info[2]
// (forced if > 0, else max(64, 8 * mean degree)), info[4] = the largest of
// their degrees; info[1] and info[4] must be zero.
hipError_t launch_heavy_list(int32_t n, const int32_t *row_ptr, int32_t forced, int32_t *heavy, int32_t *info,
                             hipStream_t s);
// Small graphs (words == 1, msbfs_fused_lds_bytes(n) of LDS): every level of
// each group in one workgroup, replacing init + the per-level launches; the
// planes must be zero beforehand.  group_out[2g] = last level with new
// vertices, group_out[2g + 1] = hop-range flag.
size_t msbfs_fused_lds_bytes(int32_t n);
hipError_t launch_msbfs_fused(const MsbfsArgs &a, int L_cap, bool full_hops, int32_t *group_out, hipStream_t s);
// The same search with the CSR and a 64-source hop tile in LDS
// (msbfs_fused_rows_lds_bytes(n, nnz) bytes): writes each group's hop rows
// to hop_out + hop_row[slot] * row_stride and the per-slot counts of hops
// 1..16 to part[slot * 16 + h - 1] (the layout launch_knn_select_counted
// reads with chunks = 1) instead of bit-planes; group_out as above.
size_t msbfs_fused_rows_lds_bytes(int32_t n, int32_t nnz);
hipError_t launch_msbfs_fused_rows(const MsbfsArgs &a, int L_cap, bool full_hops, int32_t nnz, uint8_t *hop_out,
                                   const int64_t *hop_row, int64_t row_stride, unsigned int *part,
                                   int32_t *group_out, hipStream_t s);
// One BFS level: commit the previous level's frontier, then find level `level`.
// commit_only: only commit (used after the last level the caller wants).
// Level 1 (commit of the sources, hop-1 frontier) as a fill of visited and
// the next frontier plus a per-source scatter of the sources' bits to their
// neighbours; leaves the same state and level-1 new-bit counts as
// launch_msbfs_level(a, 1, false, s).  The level-1 counters must be zero.
hipError_t launch_msbfs_first(const MsbfsArgs &a, hipStream_t s);
hipError_t launch_msbfs_level(const MsbfsArgs &a, int level, bool commit_only, hipStream_t s);
// The top-down form of level `level` (2 <= level <= a.push_levels) for the
// groups that pick it; launched beside launch_msbfs_level, whose blocks of
// those groups return at once (and the other way round).
hipError_t launch_msbfs_push(const MsbfsArgs &a, int level, hipStream_t s);
// After levels [first, last) of a round: out[0] = bit_length of the last
// level that found vertices (the plane count the transpose needs once the
// BFS is complete), out[1] = 1 if level last - 1 still found vertices.
hipError_t launch_msbfs_depth(const MsbfsArgs &a, int first, int last, int32_t *out, hipStream_t s);
// Hop rows of this round's slots: hop_out + slot_row[slot] * row_stride
// receives the n hop bytes of that slot (planes_used bit-planes committed).
hipError_t launch_msbfs_hops(const MsbfsArgs &a, int planes_used, uint8_t *hop_out,
                             const int64_t *slot_row, int64_t row_stride, hipStream_t s);
// Same, also writing per-slot counts of vertices at hops 1..16, one partial
// count per block of vertex tiles: part[(local_slot * chunks + c) * 16 + h - 1]
// with chunks = msbfs_hop_chunks(n, groups).
int msbfs_hop_chunks(int32_t n, int32_t groups);
hipError_t launch_msbfs_hops_counted(const MsbfsArgs &a, int planes_used, uint8_t *hop_out,
                                     const int64_t *slot_row, int64_t row_stride,
                                     unsigned int *part, hipStream_t s);
// Aggregated stress of a drawing over the round's hop rows, fused into the
// transpose (no rows written): per (local slot, block c) the FP64 sum of
// ((h - |X_s - X_v|) / h)^2 over v with 1 <= h <= 254 and the number of such
// v, at [local_slot * chunks + c] with chunks = msbfs_hop_chunks(n, groups).
struct StressArgs {
    const float2 *xy;          // drawing, one (x, y) per vertex
    double *part_sum;
    unsigned int *part_pairs;
};
hipError_t launch_msbfs_stress(const MsbfsArgs &a, int planes_used, const StressArgs &sa, hipStream_t s);

// ------------------------------------------------ drawing quality metrics ---
// Neighbourhood preservation (r = 1 or 2) of the drawing xy (x, y per vertex)
// for the listed vertices (all when verts is NULL): score[i] (FP64, NaN for
// an empty ball) and, when ball is not NULL, ball[i] = |N_G(v, r)|.  The
// kernel keeps an n-bit set in LDS: neighborhood_lds_bytes(n) dynamic bytes.
// evals (optional, device) accumulates the squared distances evaluated.
size_t neighborhood_lds_bytes(int32_t n);
hipError_t launch_neighborhood(int32_t n, const int32_t *row_ptr, const int32_t *col, const float *xy, int r,
                               const int32_t *verts, int32_t n_verts, double *score, int32_t *ball,
                               unsigned long long *evals, hipStream_t s);

// ------------------------------------------------------- kNN selection ---
// Rows: for r in [0, rows): hop row hop_rows + row_of[r] * row_stride (n bytes),
// source vertex src_of[r]; writes ids/hops rows out_row[r].
hipError_t launch_knn_select(int32_t n, int32_t k, int32_t rows, const uint8_t *hop_rows,
                             const int64_t *row_of, int64_t row_stride, const int32_t *src_of,
                             const int64_t *out_row, int32_t *ids, uint8_t *hops, hipStream_t s);
// Same, with the per-block counts of vertices at hops 1..16 written by
// launch_msbfs_hops_counted (part, `chunks` blocks per row); used when k <= 16.
// With the canonical CSR (csr_row_ptr, csr_col; may be null) and src_of[r] the
// source vertex of row r, the entries at hop 1 are copied from the source's
// adjacency row instead of found in the hop row.
hipError_t launch_knn_select_counted(int32_t n, int32_t k, int32_t rows, const uint8_t *hop_rows,
                                     const int64_t *row_of, int64_t row_stride, const int32_t *src_of,
                                     const int64_t *out_row, const unsigned int *part, int32_t chunks,
                                     const int32_t *csr_row_ptr, const int32_t *csr_col,
                                     int32_t *ids, uint8_t *hops, hipStream_t s);

// Copy output rows src_row -> dst_row for repeated sources (pairs on device).
hipError_t launch_copy_rows(int32_t pairs, const int64_t *dst_src, int32_t k, int32_t n,
                            int32_t *ids, uint8_t *hops, uint8_t *hop_matrix, hipStream_t s);

// ---------------------------------------------------------- partial BFS ---
struct PartialArgs {
    int32_t k;
    // single graph
    int32_t n;
    const int32_t *row_ptr;
    const int32_t *col;
    // outputs (rows indexed by vertex)
    int32_t *ids;
    uint8_t *hops;
    float *weights;           // optional fused membership (may be NULL)
    float *rho;
    float *sigma;
};
hipError_t launch_partial_bfs(const PartialArgs &a, hipStream_t s);

// Batched form: packed graphs, persistent waves pulling vertex chunks.
struct BatchArgs {
    int32_t k;
    int32_t n_graphs;
    int64_t total_vertices;
    const int64_t *vtx_offset;
    const int64_t *edge_offset;
    const int32_t *row_ptr;
    const int32_t *col;
    int32_t *ids;
    uint8_t *hops;
    float *weights;
    float *rho;
    float *sigma;
    unsigned long long *work_counter;  // zeroed by launch_batch_reset
    int32_t chunk;            // vertices taken per grab (<= batch_chunk_rows(k))
    int32_t waves_per_block;
    int32_t blocks;
    int32_t lanes;            // lanes per source: 16, 32 or 64 (k + 1 <= lanes), -1 a wave with LDS state, 0 automatic
};
hipError_t launch_batch_reset(unsigned long long *counter, hipStream_t s);
hipError_t launch_partial_batch(const BatchArgs &a, hipStream_t s);
// Largest chunk (rows per grab) the batch/jobs kernels accept for this k.
int batch_chunk_rows(int k);
// Lanes-per-source settings valid for this k (16, 32, 64 where k + 1 fits, and
// -1 for the LDS form); returns how many were written to out (at most 4).
int partial_lane_options(int k, int32_t *out);

// Served form: resident jobs and the chunks of rows of one device iteration.
struct DevJob {
    const int32_t *row_ptr;   // canonical CSR of the job
    const int32_t *col;
    int32_t n, k;
    int32_t *ids;
    uint8_t *hops;
    float *weights;           // NULL: no membership
    float *rho;
    float *sigma;
};
struct JobChunk {
    int32_t job;              // index into the job table
    int32_t begin, end;       // rows [begin, end), end - begin <= batch_chunk_rows(k)
    int32_t pad;
};
hipError_t launch_partial_jobs(const DevJob *jobs, const JobChunk *chunks, int32_t n_chunks, int max_k,
                               unsigned long long *counter, int blocks, hipStream_t s);
// Co-resident blocks of the batch kernel on the current device.
int partial_batch_max_blocks();

// ---------------------------------------------------- layout step (C2) ---
// Fuzzy union of a directed kNN membership graph (rows x k cells) into a
// symmetric CSR; *nnz (device) receives the entry count, entries beyond
// `cap` are not stored.  err (device) gets bit 1 for an id out of range or
// equal to its row.  scratch: union_scratch_bytes(rows, k, &tmp).
size_t union_scratch_bytes(int32_t rows, int32_t k, size_t *sort_tmp);
hipError_t launch_fuzzy_union(int32_t rows, int32_t k, const int32_t *ids, const float *w, int32_t *row_ptr,
                              int32_t *col, float *val, int64_t cap, int64_t *nnz, int *err, void *scratch,
                              hipStream_t s);
// E_k of a CSR (m = row_ptr[n] entries) ordered by (SplitMix64 key of the
// entry position, position).  scratch: shuffle_scratch_bytes(m, &tmp).
size_t shuffle_scratch_bytes(int64_t m, size_t *sort_tmp);
hipError_t launch_edge_shuffle(int32_t n, int64_t m, const int32_t *row_ptr, const int32_t *col, const float *val,
                               uint64_t seed, int32_t *head, int32_t *tail, float *w, void *scratch, hipStream_t s);
// GradSample windows over a shuffled edge array.  Positions are fixed point
// (int64, 2^-32 units) in two alternating buffers of 2 n values.
constexpr double kLayoutCoordLimit = 1048576.0;   // |coordinate| < 2^20 keeps P * 2^-32 exact in FP64
constexpr int kLayoutHeavyInc = 64;               // incidences above which a vertex gets a whole wave
struct LayoutArgs {
    int32_t n;
    int64_t m;                // edges in the array
    int64_t s;                // window (edges per iteration), 1 <= s <= m
    const int32_t *head;
    const int32_t *tail;
    const float *w;
    double alpha, beta;       // curve w = 1 / (1 + alpha d^(2 beta))
    double att_num;           // (-2 alpha) beta
    double rep_num;           // (2 gamma) beta
    int32_t neg;              // negative samples per edge
    uint64_t seed;            // seed of the negative samples
    // incidence lists (launch_layout_incidence)
    const int32_t *off;       // n + 1 offsets into rec
    const uint32_t *code;     // position << 1 | role (0 head, 1 tail) of each incidence, 2 m codes
    const int32_t *heavy;     // vertices with more than kLayoutHeavyInc incidences
    const int32_t *n_heavy;   // their count (device)
    int32_t heavy_blocks;     // blocks of the window launch given to heavy vertices
};
// err bit 1: head or tail outside [0, n).
hipError_t launch_edge_check(int32_t n, int64_t m, const int32_t *head, const int32_t *tail, int *err, hipStream_t s);
// p0 = round(xy * 2^32), p1 = 0; err bit 2: a coordinate not finite or not below 2^20 in magnitude.
hipError_t launch_layout_init(int32_t n, const float *xy, long long *p0, long long *p1, int *err, hipStream_t s);
hipError_t launch_layout_out(int32_t n, const long long *p, float *xy, hipStream_t s);
// Incidence lists of g's edge array (fills g.off, g.code, g.heavy, g.n_heavy;
// the caller sets g.heavy_blocks, normally to the heavy count read back).  off: n + 1 ints, code: 2 m codes, heavy: n ints,
// n_heavy: one int; scratch: incidence_scratch_bytes(n, m, &tmp).
size_t incidence_scratch_bytes(int32_t n, int64_t m, size_t *sort_tmp);
hipError_t launch_layout_incidence(LayoutArgs &g, void *scratch, int32_t *off, uint32_t *code, int32_t *heavy,
                                   int32_t *n_heavy, hipStream_t s);
// Window entries l0 .. l1 - 1 of iteration `it` (one synchronous part of the
// window) at learning rate lr: reads the positions R, writes N; moves: 32
// bytes per array position (m entries).
hipError_t launch_grad_window(const LayoutArgs &g, int32_t it, int64_t l0, int64_t l1, double lr, const long long *R,
                              long long *N, void *moves, hipStream_t s);

// -------------------------------------------- spectral initial drawing ---
// Lanczos iteration on A = D^-1/2 W D^-1/2 deflated by D^1/2 1 (FP64).
struct SpectralArgs {
    int32_t n;
    const int32_t *row_ptr;   // symmetric weighted CSR
    const int32_t *col;
    const float *val;
    double *sinv;             // n: 1 / sqrt(degree)
    double *Q;                // column-major basis, ld doubles per column; column 0 = D^1/2 1 normalised
    size_t ld;
    double *w;                // n: work vector
    double *part;             // spectral_tiles(n) x (columns + 2) partial sums
    double *h, *hacc;         // projections of the current step (columns + 2)
    double *alpha, *beta;     // recurrence coefficients, index = step (columns + 2)
    double *scal;             // 8 scalars
    double *X;                // 2 n: the two Ritz vectors, column-major
    double tiny;              // norms at or below this count as zero (Krylov space exhausted)
    int32_t *heavy;           // n: rows with many entries (one block each in the sparse product)
    int32_t heavy_rows;       // their count (read back after the setup)
};
int spectral_tiles(int32_t n);
// Degrees (err bit 1: zero degree, bit 2: a weight negative or not finite),
// column 0 = D^1/2 1 normalised, and the list of long rows (a.heavy,
// *heavy_count entries; *heavy_count zero beforehand).
hipError_t launch_spectral_setup(const SpectralArgs &a, int *err, int32_t *heavy_count, hipStream_t s);
// Column c0: the first Lanczos vector, from a SplitMix64-seeded vector
// orthogonalised against columns 0 .. c0 - 1.
hipError_t launch_lanczos_start(const SpectralArgs &a, int c0, uint64_t seed, hipStream_t s);
// Step j >= 1 (vector j in column c0 + j - 1): the next column, alpha[j] and
// beta[j] (0 when the Krylov space is exhausted).
hipError_t launch_lanczos_step(const SpectralArgs &a, int c0, int j, hipStream_t s);
// X[:, k] = Q[:, c0 .. c0 + m) svec (svec: m doubles on the device).
hipError_t launch_ritz_vector(const SpectralArgs &a, int c0, int m, const double *svec, int k, hipStream_t s);
// Q[:, col] = X[:, k] normalised.
hipError_t launch_ritz_deflate(const SpectralArgs &a, int k, int col, hipStream_t s);
// The two columns of X normalised, signed and scaled into xy (float, x y
// per vertex); first: two ints set to INT32_MAX beforehand.
hipError_t launch_spectral_finish(const SpectralArgs &a, int *first, float *xy, hipStream_t s);
// Host: largest eigenvalue of a symmetric tridiagonal matrix (diagonal a[0..m),
// off-diagonal b[0..m-1)) and its unit eigenvector z[0..m); false on failure.
bool tridiag_top(int m, const double *a, const double *b, double *theta, double *z);

// ----------------------------------------------- spectral sparsification ---
struct SparsifyArgs {
    int32_t n;
    int64_t m;                // undirected edges (read back after launch_edge_ids)
    const int32_t *row_ptr;   // canonical symmetric CSR
    const int32_t *col;
    int32_t *upper;           // n + 1: edges per row (reused for output counts)
    int32_t *eoff;            // n + 1: first edge of each row
    int32_t *eid;             // nnz: edge of each entry (-1: self-loop or unmatched)
    int32_t *eu, *ev;         // m: the edges (u < v) in CSR order
    double *B, *X, *Rv, *Z, *P, *AP;   // n x q each, row-major
    double *part;             // sparsify_tiles(n) x q x 3
    double *sums;             // q x 3
    double *st;               // q x 8: CG scalars per column
    int *active;              // q: 1 running, 2 stopping now, 0 stopped
    int *n_active;
    int32_t *comp, *parent;   // n
    int32_t *bestE;           // n
    unsigned long long *bestR;  // n
    unsigned long long *vkey;   // n: each vertex's best edge key in a forest round
    int32_t *ve;              // n: and that edge
    uint8_t *keep;            // m
};
int sparsify_tiles(int32_t n);
// upper, eoff (exclusive scan, scan_tmp: exclusive_scan_scratch_bytes(n)), eid, eu, ev.
hipError_t launch_edge_ids(const SparsifyArgs &a, void *scan_tmp, hipStream_t s);
// Right-hand sides B^T s_k (k < q, signs from SplitMix64(seed, k m + e + 1)),
// CG start (x = 0) and the per-column state; active columns get 1.
hipError_t launch_resistance_setup(const SparsifyArgs &a, int32_t q, uint64_t seed, double tol, hipStream_t s);
// One preconditioned CG iteration of every active column; *n_active = columns still running.
hipError_t launch_cg_iteration(const SparsifyArgs &a, int32_t q, double tol, int max_iters, hipStream_t s);
hipError_t launch_resistance_out(const SparsifyArgs &a, int32_t q, double *R, hipStream_t s);
// Maximum spanning forest by (R descending, edge ascending): init, then
// rounds until a round adds no edge (*added: edges of the round, zero it first).
hipError_t launch_forest_init(const SparsifyArgs &a, hipStream_t s);
hipError_t launch_forest_round(const SparsifyArgs &a, const double *R, int *added, hipStream_t s);
// The `need` best edges outside the forest join it (scratch: rank_scratch_bytes(m, &tmp)).
size_t rank_scratch_bytes(int64_t m, size_t *sort_tmp);
hipError_t launch_take_top(const SparsifyArgs &a, const double *R, int64_t need, void *scratch, hipStream_t s);
// CSR of the kept edges (both directions, columns in the input order).
hipError_t launch_sparsified_csr(const SparsifyArgs &a, int32_t *out_rp, int32_t *out_col, void *scan_tmp,
                                 hipStream_t s);

// ----------------------------------------------------------- membership ---
hipError_t launch_membership(int32_t rows, int32_t k, const uint8_t *hops, float *weights,
                             float *rho, float *sigma, hipStream_t s);

}  // namespace gm
