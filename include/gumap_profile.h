/*
 * gumap kernel timing (instrumentation of the library's own launches; not a
 * step of the method).
 *
 * When enabled, every kernel launch the library makes is bracketed by two
 * HIP events recorded on the stream the kernel is launched on, and tagged
 * with the algorithmic bytes that launch moves (the bytes its traversal
 * must read and write, computed from the sizes and from the device-side
 * work counters of the BFS levels); for the FP64 kernels "neighborhood"
 * and "msbfs_stress" the figure is their FP64 operation count instead.  Timings are resolved when a call
 * returns, so they cover exactly the calls made while enabled.  Not thread
 * safe against concurrent library calls from several threads.
 */
#ifndef GUMAP_PROFILE_H
#define GUMAP_PROFILE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Starts (on != 0) or stops recording.  Recording adds two event records per launch. */
void gumap_profile_enable(int on);
/* Restricts recording to the kernels named in `names`, a comma-separated
 * list of the names gumap_profile_entry reports (say "msbfs_level"); NULL or
 * "" records every kernel again.  The list is copied.  Launches of other
 * kernels then get no events, so they run as with recording off. */
void gumap_profile_only(const char *names);
/* Drops everything recorded so far. */
void gumap_profile_reset(void);
/* Number of distinct kernels recorded. */
int gumap_profile_count(void);
/* Entry i (0 <= i < count): kernel name (owned by the library), number of
 * launches, total elapsed milliseconds and total algorithmic bytes.
 * Returns 0, or -1 if i is out of range. */
int gumap_profile_entry(int i, const char **name, int64_t *launches, double *total_ms,
                        double *alg_bytes);
/* Entry i's total bytes moved beyond its algorithmic bytes: for "msbfs_level"
 * the lazy commit of the previous level (the visited word written back and
 * the bit-plane read-modify-writes of each committed word), which the
 * per-level byte count of the all-source BFS does not include; 0 for other
 * kernels.  Returns 0, or -1 if i is out of range. */
int gumap_profile_extra(int i, double *extra_bytes);

#ifdef __cplusplus
}
#endif

#endif /* GUMAP_PROFILE_H */
