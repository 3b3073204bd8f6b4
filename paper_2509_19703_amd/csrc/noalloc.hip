// gumap_knn_partial_noalloc: the partial-BFS kNN (Sec. 3.3.1, Alg. 4) for
// callers that cannot allocate (code under HIP graph capture, tight serving
// loops).  It runs the kernels of gumap_knn_partial, and the canonical CSR
// and the canonicalisation's work arrays live in one fixed device array,
// `scratch`, instead of the library's grow-only cache.
//
// `scratch` is a file-scope __device__ array: every device the library runs
// on holds its own copy at its own address for the life of the process.  Its
// name in host code is only a host-side stand-in, so the device address is
// looked up once per device (hipGetSymbolAddress, with that device current)
// and kept; only that address is passed to kernels.  Every call on a device
// shares the array: calls that overlap on one device race.  Nothing in it
// needs to start at zero (the canonicalisation writes every word it reads).
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "kernels.h"
#include "runtime.h"

namespace {

static __device__ __align__(256) unsigned char scratch[GUMAP_NOALLOC_SCRATCH_BYTES];

constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct NoallocScratch {
    void *ptr = nullptr;
};

NoallocScratch &noalloc_of(int dev)
{
    static NoallocScratch per_dev[64];
    return per_dev[dev & 63];
}

// The current device's address of `scratch` (looked up on the first call on
// that device).
int noalloc_scratch(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return gm::hip_status(e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return gm::set_error(GUMAP_EINVAL, "device %d beyond the 64 the library tracks", dev);
    NoallocScratch &d = noalloc_of(dev);
    if (!d.ptr) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return gm::set_error(GUMAP_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                                 hipGetErrorString(e));
        }
        d.ptr = p;
    }
    *out = d.ptr;
    return GUMAP_OK;
}

int knn_partial_noalloc(const gumap_graph *g, int32_t k, int32_t *ids, uint8_t *hops, hipStream_t s)
{
    int st;
    if ((st = gm::check_graph_args(g))) return st;
    if ((st = gm::check_k(k))) return st;
    if (g->flags & GUMAP_VALIDATE)
        return gm::set_error(GUMAP_EINVAL, "GUMAP_VALIDATE is not accepted without allocation (its result is read "
                                           "back through pinned host memory the library allocates)");
    if (g->n > 0 && (!ids || !hops)) return gm::set_error(GUMAP_EINVAL, "output pointer is NULL");
    if (g->n == 0) return GUMAP_OK;
    const int32_t n = g->n, nnz = g->nnz;
    const int32_t *rp = g->row_ptr, *col = g->col_idx;
    hipError_t e;
    if (!(g->flags & GUMAP_CSR_SORTED)) {
        const size_t rp_bytes = align256((size_t)(n + 1) * sizeof(int32_t));
        const size_t col_bytes = align256((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
        const size_t need = rp_bytes + col_bytes + gm::canon_scratch_bytes(n, nnz);
        if (need > (size_t)GUMAP_NOALLOC_SCRATCH_BYTES)
            return gm::set_error(GUMAP_E2BIG, "graph needs %zu bytes of scratch; the no-allocation maximum is %zu "
                                              "(canonicalise it once and pass GUMAP_CSR_SORTED)",
                                 need, (size_t)GUMAP_NOALLOC_SCRATCH_BYTES);
        void *base = nullptr;
        if ((st = noalloc_scratch(&base))) return st;
        char *p = (char *)base;
        int32_t *crp = (int32_t *)p;
        int32_t *ccol = (int32_t *)(p + rp_bytes);
        void *tmp = p + rp_bytes + col_bytes;
        e = gm::launch_canonicalize(n, nnz, rp, col, crp, ccol, tmp, s);
        if (e != hipSuccess) return gm::hip_status(e, "canonicalize");
        rp = crp;
        col = ccol;
    }
    gm::PartialArgs a{};
    a.k = k;
    a.n = n;
    a.row_ptr = rp;
    a.col = col;
    a.ids = ids;
    a.hops = hops;
    e = gm::launch_partial_bfs(a, s);
    if (e != hipSuccess) return gm::hip_status(e, "partial bfs");
    e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipGetLastError();
    return gm::hip_status(e, "gumap_knn_partial_noalloc");
}

}  // namespace

extern "C" int gumap_knn_partial_noalloc(const gumap_graph *g, int32_t k, int32_t *nbr_ids, uint8_t *nbr_hops,
                                         hipStream_t stream)
{
    std::lock_guard<std::mutex> lock(gm::api_mutex());
    gm::clear_error();
    int st = knn_partial_noalloc(g, k, nbr_ids, nbr_hops, stream);
    if (st != GUMAP_OK && st != GUMAP_EINVAL) {
        (void)hipStreamSynchronize(stream);
        (void)hipGetLastError();
    }
    return st;
}
