// Host-side runtime shared by the C-ABI entry points and the request server:
// per-device cached scratch, error reporting and the internal call bodies.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <stddef.h>
#include <stdint.h>

#include "../../include/gumap.h"

namespace gm {

// Scratch slots: each is a grow-only device buffer per device.
enum ScratchSlot {
    kSlotFlags = 0,
    kSlotCanonRp,
    kSlotCanonCol,
    kSlotCanonTmp,
    kSlotUsrc,
    kSlotSlotOf,
    kSlotSlotRow,
    kSlotDup,
    kSlotBfsState,
    kSlotStats,
    kSlotLvlCnt,
    kSlotHopRows,
    kSlotLocalRows,
    kSlotUnionRp,
    kSlotUnionCol,
    kSlotBatchEoff,
    kSlotBatchRp,
    kSlotBatchCol,
    kSlotCounter,
    kSlotHeavy,
    kSlotStressSum,
    kSlotStressPairs,
    kSlotEvals,
    kSlotInfo,
    kSlotFirst,
    kSlotMarks,
    kSlotPos,
    kSlotScanTmp,
    kSlotCount,
    kSlotMult,
    kSlotGroupOut,
    kSlotUnion,
    kSlotShuffle,
    kSlotLayoutPos,
    kSlotLayoutSort,
    kSlotLayoutRec,
    kSlotLayoutMoves,
    kSlotSpectral,
    kSlotSpectralVec,
    kSlotSparsify,
    kSlotSparsifyRank,
    kScratchSlots
};

struct CanonCsr {
    int32_t n = 0;
    const int32_t *row_ptr = nullptr;
    const int32_t *col = nullptr;
};

int set_error(int status, const char *fmt, ...);
void clear_error();
const char *last_error();
int hip_status(hipError_t e, const char *what);
std::mutex &api_mutex();
size_t env_size(const char *name, size_t dflt);

// Launch settings of the all-source BFS (gumap_knn_build, gumap_stress) that
// change only its speed; -1 leaves a setting to its default.  A setting
// given in the environment (GUMAP_FUSED, GUMAP_FORCE_WORDS,
// GUMAP_LEVEL_VERTS, GUMAP_FIRST_LEVEL, GUMAP_HEAVY_DEGREE,
// GUMAP_HIST_LEVELS, GUMAP_PUSH_LEVELS) takes precedence.
struct BuildKnobs {
    int fused = -1;    // 1: one workgroup per group runs every level (small graphs); 0: per-level launches
    int words = -1;    // 64-bit source words per vertex per group: 1, 2, 4, 8
    int verts = -1;    // (vertex, word) items per thread of the level kernel: 1, 2, 4, 8
    int first = -1;    // level 1: 1 fill + top-down scatter, 0 range scan in the level kernel
    int heavy = -1;    // degree above which a vertex is searched by a whole wave; 0: the default rule
    int hist = -1;     // hops kept as frontiers instead of bit-planes (0: planes only)
    int push = -1;     // levels that may run top-down (0: bottom-up only)
};
// The value of knob `name`: the environment's if set, else kb_value if >= 0, else dflt.
size_t knob(const char *name, int kb_value, size_t dflt);
int knn_build_tuned(const gumap_graph *g, int32_t k, const int32_t *sources, int32_t n_sources, int32_t *ids,
                    uint8_t *hops, uint8_t *hop_matrix, hipStream_t s, const BuildKnobs *kb);
// The settings the autotuner recorded for calls of this shape, if any.
bool tuned_knobs(int32_t n, int64_t nnz, int64_t rows, int32_t k, bool hop_matrix, BuildKnobs *out);

int scratch_get(int slot, size_t bytes, void **out);
int host_scratch_get(size_t bytes, void **out);

int check_graph_args(const gumap_graph *g);
int check_k(int32_t k);
int prepare_graph(const gumap_graph *g, hipStream_t s, CanonCsr *out);
int check_batch_args(const gumap_batch *b, int32_t k);
int prepare_batch(const gumap_batch *b, hipStream_t s, gumap_batch *out);
// Launch configuration of the batch kernel; zero fields take the defaults.
struct BatchTune {
    int32_t lanes = 0, chunk = 0, blocks = 0;
};
// Enqueues the batched partial BFS (+ membership when w != NULL) of a
// canonical packed batch with configuration t (NULL: defaults); no
// synchronisation.
int batch_enqueue(const gumap_batch *b, int32_t k, int32_t *ids, uint8_t *hops, float *w, float *rho,
                  float *sigma, hipStream_t s, const BatchTune *t = nullptr);

}  // namespace gm
