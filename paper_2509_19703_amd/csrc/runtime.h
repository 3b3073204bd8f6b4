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
