/*
 * qfs.h -- C ABI of libqfs: quasi-F-split (Artin-Mazur) heights of quartic
 * K3 surfaces over F_p on AMD Instinct MI355X (gfx950).
 *
 * Method: Batubara, Garzella, Pan, "K3 surfaces of any Artin-Mazur height
 * over F5 and F7 via quasi-F-split singularities and GPU acceleration"
 * (arXiv 2502.12428).  For a quartic f in F_p[x1,x2,x3,x4]:
 *   g     = f^(p-1) mod p                       (Algorithm 3, first line)
 *   h = 1 if g is not in m^[p]                   (Fedder's criterion, Section 2.2)
 *   Delta = Delta_1(g) = (g~^p - sum_t t^p)/p    (Algorithm 1, Section 3.1)
 *   theta(a) = u(Delta * a)                      (Algorithm 2 and Section 3.4)
 *   h = least k in 2..bound with theta^(k-1)(g) not in m^[p], else infinity
 *                                                (Algorithm 3; Theorem C with h <= 10 for K3)
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Coefficient arrays are uint8, one value in [0, p) per monomial, row-major
 *   [batch][len].  A homogeneous form of degree n has len = C(n+3, 3)
 *   monomials (Section 4, Lemma "wics size"), stored in descending
 *   lexicographic order of the exponent tuple (e1,e2,e3,e4), x1 > x2 > x3 > x4
 *   (the order the paper's tables print terms in).  The position of (e1..e4)
 *   is qfs_monomial_rank(e) = C(e2+e3+e4+2,3) + C(e3+e4+1,2) + e4.
 *   A quartic is 35 bytes; g has C(4p-1,3) bytes; Delta has C(4p(p-1)+3,3).
 * - Supported primes: 3, 5, 7, 11.
 * - Array arguments marked "device" are device pointers, allocated and owned
 *   by the caller (e.g. the data_ptr() of a torch tensor).  The library never
 *   allocates device memory: scratch comes from the caller's workspace `ws`,
 *   which must be 256-byte aligned and hold at least the bytes reported by the
 *   matching *_workspace_bytes() call; its contents need no initialisation
 *   and are clobbered.
 * - Calls are asynchronous on `stream` (0 = the null stream): they enqueue
 *   kernels and return.  Argument errors are detected on the host before
 *   anything is enqueued and are returned as a negative qfs_status; the text
 *   is available from qfs_last_error() in the calling thread.
 * - Calls that share a workspace must not overlap in time.
 */
#ifndef QFS_H
#define QFS_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QFS_OK = 0,
    QFS_EINVAL = -1,      /* bad argument (null pointer, size, bound, coefficient >= p) */
    QFS_ENOMEM = -2,      /* workspace smaller than required */
    QFS_EDEVICE = -3,     /* a HIP runtime call failed */
    QFS_EUNSUPPORTED = -4,/* prime not in {3, 5, 7, 11} */
    QFS_EARITH = -5       /* an internal exactness check failed (never expected) */
} qfs_status;

/* Height value meaning "infinite" (no height <= bound); finite heights are 1..bound. */
#define QFS_HEIGHT_INF 0

/* Number of monomials of degree deg in 4 variables: C(deg+3, 3); 0 if deg < 0. */
int64_t qfs_num_monomials(int deg);

/* Position of the exponent tuple e[0..3] (host pointer) in its degree's
 * coefficient array (formula above); -1 if some exponent is negative. */
int64_t qfs_monomial_rank(const int32_t e[4]);

/* Inverse of qfs_monomial_rank for degree deg: writes e[0..3] (host pointer).
 * Returns QFS_OK, or QFS_EINVAL if rank is outside [0, qfs_num_monomials(deg)). */
int qfs_monomial_unrank(int deg, int64_t rank, int32_t e[4]);

/* Coefficient counts for prime p: len of g = C(4p-1,3), len of Delta = C(4p(p-1)+3,3). */
int64_t qfs_len_g(int p);
int64_t qfs_len_delta(int p);

/* ------------------------------------------------------------------------
 * qfs_delta1 -- Algorithm 1 applied to g = f^(p-1) (Section 3.1,
 * Proposition "delta1 formula"; Algorithm 3, lines 1 and 4).
 *
 *   f          device, [batch][35], values in [0,p): the quartics.
 *   g_out      device, [batch][C(4p-1,3)] or NULL: receives g = f^(p-1) mod p.
 *   delta_out  device, [batch][C(4p(p-1)+3,3)]: receives Delta_1(g) mod p,
 *              with the sign of Algorithm 1: (g~^p - sum_t t^p)/p, where g~
 *              lifts g with coefficients in [0,p) and t runs over its terms.
 *   status_out device, [batch] int32 or NULL: per-surface QFS_OK, or
 *              QFS_EINVAL if some coefficient of f is >= p (outputs of that
 *              surface are then unspecified), or QFS_EARITH.
 * g~^p is formed in Z/p^2 on int8 matrix cores with int32 accumulation; the
 * Delta_1 division is exact and checked.
 * Returns QFS_OK or a negative qfs_status (nothing enqueued on error).
 * ---------------------------------------------------------------------- */
size_t qfs_delta1_workspace_bytes(int p, int batch);
int qfs_delta1(int p, int batch, const uint8_t *f, uint8_t *g_out, uint8_t *delta_out,
               int32_t *status_out, void *ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * qfs_theta -- iterate the "multiply then split" map theta(a) = u(Delta a)
 * (Algorithm 2 applied to Delta*a; Section 3.4): out = theta^iters(a).
 *
 *   delta  device, [batch][C(4p(p-1)+3,3)], values in [0,p): Delta per surface.
 *   a      device, [batch][C(4p-1,3)], values in [0,p): the starting forms.
 *   out    device, [batch][C(4p-1,3)]: theta^iters(a); may not alias a.
 *   iters  0..64 (0 copies a).
 * Values >= p in delta or a are the caller's error; they are reduced mod p.
 * ---------------------------------------------------------------------- */
size_t qfs_theta_workspace_bytes(int p, int batch);
int qfs_theta(int p, int batch, const uint8_t *delta, const uint8_t *a, uint8_t *out, int iters,
              void *ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * qfs_height -- Algorithm 3 for a batch of quartics over possibly different
 * primes, in one batched launch sequence (surfaces grouped by p; only those
 * that fail Fedder's criterion run Delta_1 and theta).
 *
 *   batch    number of surfaces (0 is allowed and enqueues nothing).
 *   p        device, [batch] int32: each surface's prime.
 *   f        device, [batch][35], values in [0,p).
 *   bound    1..10: the b of Algorithm 3 (10 for K3 surfaces).
 *   max_p    the largest prime the batch may hold (3, 5, 7 or 11); it sizes
 *            the workspace, and surfaces with a larger p are rejected.
 *   heights  device, [batch] int32: 1..bound, QFS_HEIGHT_INF (0), or a
 *            negative qfs_status for that surface (QFS_EUNSUPPORTED for a
 *            prime outside {3,5,7,11} or above max_p, QFS_EINVAL for a
 *            coefficient >= p, QFS_EARITH for a failed exactness check).
 * The workspace must hold qfs_height_workspace_bytes(batch, max_p) bytes.
 * Launches: Fedder's test, g for the deep surfaces, then per prime the
 * capped-chain kernel and the full-chain kernel.  With option "height_graph"
 * (default on) the whole sequence is captured into a hipGraph the second
 * time an argument set (every pointer and size) is met, up to 8 cached with
 * the least recently used evicted, and later calls with the same arguments
 * replay it on `stream`; the library
 * holds these graphs until qfs_shutdown().  While stage timing is enabled the
 * sequence is launched directly instead.
 * ---------------------------------------------------------------------- */
size_t qfs_height_workspace_bytes(int batch, int max_p);
int qfs_height(int batch, const int32_t *p, const uint8_t *f, int bound, int max_p, int32_t *heights,
               void *ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * qfs_autotune -- times qfs_height on the caller's batch (arguments as for
 * qfs_height) over a grid of launch settings: "deep_slots" in {CUs/2,
 * 3 CUs/4, CUs} x "gpow_per_cu" in {4, 8, 16}, each after one warm-up call,
 * `reps` (1..100) timed calls, direct launches (no graphs).  It keeps the
 * fastest setting as the process-wide options and, if cache_path is not
 * NULL, appends one JSON line (device architecture, compute units, max_p,
 * batch, the chosen options, the mean milliseconds of every trial) to that
 * file.  `ws` must hold qfs_height_workspace_bytes(batch, max_p) with one
 * slot per compute unit.  heights receives the last trial's output.
 * Synchronizes `stream`.  Returns QFS_OK or a negative qfs_status (options
 * unchanged on error).
 *
 * qfs_load_tuning -- applies the last line of cache_path written by
 * qfs_autotune for this device architecture, compute-unit count and max_p.
 * Returns QFS_OK, or QFS_EINVAL if the file cannot be read or has no such line.
 * ---------------------------------------------------------------------- */
int qfs_autotune(int batch, const int32_t *p, const uint8_t *f, int bound, int max_p, int32_t *heights, void *ws,
                 size_t ws_bytes, hipStream_t stream, const char *cache_path, int reps);
int qfs_load_tuning(const char *cache_path, int max_p);

/* ------------------------------------------------------------------------
 * qfs_height_plain -- the same heights for surfaces of one prime p, computed
 * one surface at a time with plain vector-ALU kernels (no matrix cores, no
 * batching): the comparison baseline for qfs_height.  Arguments as above.
 * ---------------------------------------------------------------------- */
size_t qfs_height_plain_workspace_bytes(int p);
int qfs_height_plain(int p, int batch, const uint8_t *f, int bound, int32_t *heights,
                     void *ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * qfs_height_reduced: the same heights as qfs_height (Algorithm 3, bound
 * <= 10) from a reduced form that needs neither g~^p nor Delta_1(g).  With
 * D = Delta_1(f) (Algorithm 1 applied to f) and H = f^(p-2) mod p, the
 * binomial theorem mod p^2 gives Delta_1(f^(p-1)) = phi(Q) - D phi(H) mod p
 * (phi multiplies exponents by p); the splitting u of Algorithm 2 is
 * p^-1-linear, so along Algorithm 3's loop theta^(k-1)(g) = H v_k for quartics
 * v_1 = f, v_(k+1) = -u(D H v_k), and the test reads c(H v_k).  Not an
 * algorithm of the paper; it is checked against the paper's Algorithms 1-3
 * by the oracle tests and against qfs_height by the GPU tests.  Fedder's test
 * (Section 2.2) runs first for every surface, as in qfs_height; one
 * workgroup per remaining surface forms H and D in LDS and iterates.
 * Arguments, layouts and errors as qfs_height; the workspace is
 * qfs_height_reduced_workspace_bytes(batch, max_p) bytes (counters and one
 * queue per prime), caller-owned, 256-byte aligned.  No graph capture.
 * ---------------------------------------------------------------------- */
size_t qfs_height_reduced_workspace_bytes(int batch, int max_p);
int qfs_height_reduced(int batch, const int32_t *p, const uint8_t *f, int bound, int max_p, int32_t *heights,
                       void *ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Stage timing (diagnostics).  While enabled, every qfs_height call records
 * hipEvents on its stream around its stages; qfs_profile_collect waits for
 * the recorded events, writes the summed milliseconds per stage into
 * ms[0..QFS_PROFILE_STAGES-1] and the number of calls into *calls, and clears
 * the record.  Stages: 0 stage 1 (g and Fedder's test), 1 plans, 2..5 the
 * capped-chain launches for p = 3, 5, 7, 11, 6..9 the full-chain launches
 * (with the theta loop) for p = 3, 5, 7, 11.  Host pointers.
 * ---------------------------------------------------------------------- */
#define QFS_PROFILE_STAGES 10
int qfs_profile_enable(int on);
int qfs_profile_collect(double ms[QFS_PROFILE_STAGES], int *calls);

/* Matrix-core instructions (v_mfma_i32_16x16x64_i8, 16,384 multiply-adds
 * each) that the g~^p product issues for one surface at prime p: pass 0 is
 * the full chain (qfs_delta1, and qfs_height for surfaces of height > 2),
 * pass 1 the capped chain qfs_height runs first for every surface that fails
 * Fedder's test.  The count depends only on p and pass; -1 for an
 * unsupported p or pass. */
int64_t qfs_mfma_per_surface(int p, int pass);

/* The int8 matrix-core rate this device sustains (TOP/s, two operations per
 * multiply-add) on a loop of independent v_mfma_i32_16x16x64_i8 on register
 * operands with no memory traffic, over `iters` iterations (1..10^7) on 8
 * workgroups per compute unit: the measured ceiling for the deep kernels'
 * executed-MFMA figure, next to the nominal 5.0 POP/s.  sink: a caller-owned
 * device int the kernel may write (it does not for these operands).  Waits
 * for the measurement (hipEvents on `stream`).  Diagnostics only. */
int qfs_mfma_peak(int iters, int32_t *sink, double *tops, hipStream_t stream);

/* Process-wide options (host strings; affect calls enqueued afterwards).
 *   "height_band" (default 1): qfs_height decides h = 2 with the capped
 *     chain, which forms only the coefficients of Delta_1 that the first
 *     theta test reads (Section 3.4: c(theta(g)) = sum_c g[c] Delta[(p+1)e-c]),
 *     and runs the full chain only for surfaces of height > 2.  0 runs the
 *     full chain for every surface.  Heights are the same either way.
 *   "height_graph" (default 1): replay cached hipGraphs of the qfs_height
 *     launch sequence (see qfs_height); 0 launches the kernels directly.
 *   "height_graphs_cached" (read only): number of graphs in the cache.
 *   "chain_power_p3", "chain_power_p5", "chain_power_p7", "chain_power_p11"
 *     (read only): the power J of the deep chain's multiplier m = f~^J mod p^2
 *     at that prime.  g~^p mod p^2 (Algorithm 1) is formed as
 *     m^(p(p-1)/J) = f~^(p(p-1)), which equals g~^p mod p^2 since
 *     g~ = f~^(p-1) mod p; J = p-1 multiplies by g~ itself.
 *   "deep_slots" (default 0 = one per compute unit): persistent workgroups
 *     of the deep kernels, each with its own slot of workspace; it changes
 *     the *_workspace_bytes results, so query them after setting it.
 *   "gpow_per_cu" (default 8, 1..64): workgroups per compute unit of the
 *     kernel that forms g = f^(p-1) for the deep surfaces.
 * qfs_set_option returns QFS_OK or QFS_EINVAL (unknown name or value);
 * qfs_get_option returns the value, or QFS_EINVAL for an unknown name. */
int qfs_set_option(const char *name, int64_t value);
int64_t qfs_get_option(const char *name);

/* Message for the last error returned in the calling thread ("" if none). */
const char *qfs_last_error(void);

/* Waits for the device, then releases the graph cache and the library's
 * capture streams.  The library holds no device memory of its own. */
void qfs_shutdown(void);

#ifdef __cplusplus
}
#endif

#endif /* QFS_H */
