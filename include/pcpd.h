/*
 * pcpd.h -- C ABI of libpcpd, the MI355X (gfx950) multispin Monte Carlo sweep
 * of 1+1-dimensional reaction-diffusion models: directed percolation (DP),
 * the pair contact process with diffusion (PCPD), and the triplet and
 * quadruplet contact processes with diffusion (TCPD, QCPD), after R.D.
 * Schram, arXiv:1301.6082 (which develops the PCPD and names the others as
 * direct extensions, Sec. 1).
 *
 * What the library computes (all of it on the GPU):
 *   - The model (paper Sec. 2, eq. (1)): on a ring of L sites, attempted
 *     reactions AA0 -> AAA and 0AA -> AAA each with rate (1-p)(1-d)/2,
 *     AA -> 00 with rate p(1-d), A0 <-> 0A with rate d. The n-tuple form
 *     generalises "AA" to n particles (DP n = 1, PCPD n = 2, TCPD n = 3,
 *     QCPD n = 4).
 *   - One attempt (paper Algorithm 1): diffusion swaps sites j and j+1 with
 *     probability d; otherwise an n-tuple at j..j+n-1 annihilates with
 *     probability p, else a particle is created at j+n (R = 1, "high") or
 *     at j-1 (R = 0, "low").
 *   - Site selection (paper Sec. 3): the ring is cut into blocks of B sites;
 *     every block is attempted at one shared, uniformly drawn local site per
 *     substep; B substeps form one Monte Carlo step (time + 1).
 *   - Multispin storage (paper Sec. 4): bit b of a 64-bit word is sample b;
 *     a plane is L words (64 samples); an instance has `planes` planes.
 *   - Random numbers: Philox-4x32-10 (Salmon et al., SC'11), key
 *     (seed, stream_id), counter (k, 8*plane + draw, lo32 s, hi32 s) for
 *     window k of substep s = t*B + b; draw 7 with k = 0 gives the substep
 *     offset o = (x0 * B) >> 32. A probability-q decision of sample b is
 *     (2*bit_b(X1) + bit_b(X2)) * 2^32 + g < rint(q * 2^34), g shared by the
 *     64 samples of a word; this generalises the AND/OR masks of paper
 *     Sec. 4.2 and the shared comparison RNG() < 4p of Sec. 4.3.
 *   - Observables (paper Sec. 5.3): per (instance, plane) the particle
 *     count N, the nearest-neighbour pair count N_pair and the mask of
 *     samples that still hold a particle.
 *
 * Conventions:
 *   - Every function returns a pcpd_status (0 = success, < 0 = error); no
 *     C++ exception crosses this boundary.
 *   - Host pointers are borrowed for the duration of the call only.
 *   - Device pointers given in pcpd_device are borrowed for the lifetime of
 *     the context and must stay valid until pcpd_free.
 *   - Work is enqueued on the context's HIP stream. pcpd_sweep returns
 *     before the GPU finishes; errors of enqueued work surface at the next
 *     call that synchronises (pcpd_density, pcpd_run, pcpd_get_lattice,
 *     pcpd_sync) as PCPD_EDEVICE. After PCPD_EDEVICE the context answers
 *     PCPD_ESTATE to everything except pcpd_free.
 *   - One context must not be used from two host threads at once.
 */
#ifndef PCPD_H
#define PCPD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#ifndef PCPD_API
#define PCPD_API __attribute__((visibility("default")))
#endif

typedef enum {
    PCPD_OK = 0,
    PCPD_EINVAL = -1,     /* an argument is out of range; nothing was changed */
    PCPD_ENOMEM = -2,     /* a device or host allocation failed */
    PCPD_EDEVICE = -3,    /* a HIP call or enqueued kernel failed */
    PCPD_ESTATE = -4,     /* the context is unusable after an earlier device error */
    PCPD_EOVERFLOW = -5,  /* the substep counter t*B would leave 64 bits */
    PCPD_ELIMIT = -6      /* the problem exceeds the fixed workspace of pcpd_run_noalloc */
} pcpd_status;

typedef enum { PCPD_DP = 1, PCPD_PCPD = 2, PCPD_TCPD = 3, PCPD_QCPD = 4 } pcpd_model; /* = tuple size n */

typedef enum { PCPD_INIT_FULL = 0, PCPD_INIT_EMPTY = 1, PCPD_INIT_HOST = 2 } pcpd_init_kind;

/* Multispin layout of a plane (paper Sec. 4). */
typedef enum {
    PCPD_LAYOUT_CLASSICAL = 0, /* 64 independent rings of L sites, one per bit */
    PCPD_LAYOUT_CONNECTED = 1  /* the 64 bits joined into ONE ring of 64 L sites: site
                                  b*L + j is bit b of word j (the sites of a word are L apart),
                                  and past word L-1 of bit b comes word 0 of bit b+1 (Sec. 4,
                                  second paragraph; the layout of Figs. 2-3). The Sec. 3 scheme
                                  runs on the joined ring (64 L / B blocks); the window at site
                                  b*L + k*B + o reads bit b of word window k's draws. N_pair
                                  counts the pairs of the joined ring; alive has bit b set iff
                                  sites b*L .. b*L+L-1 hold a particle. */
} pcpd_layout;

/* Shared by all instances of a context. */
typedef struct {
    int32_t model;    /* pcpd_model */
    uint32_t B;       /* block width; B >= n+2; every L must be a multiple of B */
    uint32_t planes;  /* planes per instance, >= 1; 64 samples (or one joined ring) each */
    uint32_t seed;    /* Philox key word 0 */
    uint32_t layout;  /* pcpd_layout */
    uint32_t mask_bits; /* decorrelation bits m of every decision (Sec. 4.3): 2 (also for 0)
                           or 4. Sample b of a probability-q decision fires iff
                           u_b * 2^32 + g < rint(q * 2^(32+m)), u_b the m-bit number of bit b
                           of m independent random words and g a 32-bit part shared by the
                           word's 64 samples; m = 4 takes two more Philox draws per window.
                           Other values: PCPD_EINVAL. */
} pcpd_config;

/* One independent simulation (its own rates, ring length and Philox stream). */
typedef struct {
    double p;                   /* annihilation parameter of eq. (1), 0 <= p <= 1 */
    double d;                   /* diffusion rate of eq. (1), 0 <= d <= 1 */
    uint64_t L;                 /* ring length in sites, L >= B, L % B == 0, L/B < 2^32 */
    uint32_t stream_id;         /* Philox key word 1 */
    int32_t init;               /* pcpd_init_kind */
    const uint64_t *host_words; /* init == PCPD_INIT_HOST: planes*L words, plane-major,
                                   natural site order; otherwise ignored */
} pcpd_instance;

/* Where the library puts its work. Every field may be 0 / NULL. */
typedef struct {
    void *hip_stream;      /* hipStream_t to enqueue on; NULL = the null stream */
    void *dev_buf;         /* caller-owned device memory for the two lattice copies,
                              at least pcpd_lattice_bytes() bytes, 256-byte aligned;
                              NULL = the library allocates */
    size_t dev_buf_bytes;
} pcpd_device;

/* Counts of one (instance, plane), summed over its 64 samples. */
typedef struct {
    uint64_t n;       /* occupied sites */
    uint64_t n_pair;  /* pairs (j, j+1 mod L) with both sites occupied */
    uint64_t alive;   /* bit b set iff sample b holds at least one particle */
} pcpd_counts;

/* Kernel shape of the sweep. Results never depend on it. All three 0 = the
 * default shape (phases of at most 128 substeps, the widest tile of at most 128
 * blocks that lets two workgroups share a CU, four teams); otherwise a 0 field
 * keeps the context's current value. */
typedef struct {
    uint32_t tile_cols;  /* blocks per workgroup tile including the halo */
    uint32_t phase_max;  /* substeps run while a tile stays in LDS */
    uint32_t teams;      /* lanes per block, 2 or 4: team t applies substeps t, t+teams, ... */
} pcpd_tuning;

typedef struct pcpd_ctx pcpd_ctx;

/* Bytes of device memory for the two lattice copies of these instances
 * (2 * 8 * planes * sum L): one word per site holding 64 samples (paper
 * Sec. 4, classical multispin). Validates like pcpd_init; *bytes_out is
 * written only on success. */
PCPD_API int pcpd_lattice_bytes(const pcpd_config *cfg, const pcpd_instance *inst, uint32_t n_inst,
                       size_t *bytes_out);

/* Create a context of n_inst instances of the model of paper eq. (1) (rates
 * p, d; ring length L, Sec. 2), each started full, empty or from host words,
 * at Monte Carlo step t0. t0 > 0 resumes a stored lattice: the lattice and t
 * fully determine the future, since every random number is addressed by
 * (seed, stream_id, plane, block, substep). t0 is shared by all instances of
 * a context; instances at different times go in separate contexts.
 * Ownership: *out is library-owned until pcpd_free; cfg, inst and the host
 * words are read during the call only; dev->dev_buf (if given) is borrowed
 * for the context's lifetime. Validation failures return PCPD_EINVAL (or
 * PCPD_EOVERFLOW if t0 * B leaves 64 bits) before any device work and leave
 * *out untouched; a failed allocation returns PCPD_ENOMEM. */
PCPD_API int pcpd_init(pcpd_ctx **out, const pcpd_config *cfg, const pcpd_instance *inst,
              uint32_t n_inst, uint64_t t0, const pcpd_device *dev);

/* Advance every instance by n_steps Monte Carlo steps: paper Algorithm 1
 * (one attempt maps time t to t + 1/L) applied in the shared-local-site order
 * of Sec. 3 (every block of B sites attempted at one drawn local site per
 * substep, B substeps per step), all 64 samples of a word at once with the
 * bit masks of Sec. 4 (Algorithm 2, read so that annihilation clears the
 * tuple, l AND NOT mask, and low fission sets site j-1 itself, as Algorithm 1
 * and the prose of Sec. 4.3 state).
 * Asynchronous: errors of the enqueued kernels surface at the next
 * synchronising call. PCPD_EOVERFLOW if (t + n_steps) * B leaves 64 bits;
 * n_steps = 0 does nothing. */
PCPD_API int pcpd_sweep(pcpd_ctx *ctx, uint64_t n_steps);

/* The order parameter of paper Sec. 1 and the pair density of Sec. 5.3 for
 * the current lattice: out[i * planes + q] = (N, N_pair, alive) of instance
 * i, plane q (rho = N / (64 L)). `out` is a host array of n_inst * planes
 * entries, written only on success. Synchronises. */
PCPD_API int pcpd_density(pcpd_ctx *ctx, pcpd_counts *out);

/* Density series at scheduled times, as analysed in paper Sec. 5.3: sweep
 * (as pcpd_sweep) to each of the strictly increasing times[0..n_times) (each
 * >= the current t; a time equal to t records the current lattice) and record
 * the counts there into the host array
 * out[r * n_inst * planes + i * planes + q]. PCPD_EINVAL for unordered times
 * or a time before t (nothing is enqueued then). Synchronises once at the
 * end. */
PCPD_API int pcpd_run(pcpd_ctx *ctx, const uint64_t *times, uint32_t n_times, pcpd_counts *out);

/* Copy instance `inst`'s planes*L words (plane-major, natural order) to or
 * from the host. Synchronous. */
PCPD_API int pcpd_get_lattice(pcpd_ctx *ctx, uint32_t inst, uint64_t *host_words);
PCPD_API int pcpd_set_lattice(pcpd_ctx *ctx, uint32_t inst, const uint64_t *host_words);

/* Current Monte Carlo step. */
PCPD_API int pcpd_time(pcpd_ctx *ctx, uint64_t *t_out);

/* Wait for enqueued work and report its errors. */
PCPD_API int pcpd_sync(pcpd_ctx *ctx);

/* Set or read the kernel shape (see pcpd_tuning). PCPD_EINVAL if the shape
 * does not fit the device (LDS) or the block width. */
PCPD_API int pcpd_set_tuning(pcpd_ctx *ctx, const pcpd_tuning *tuning);
PCPD_API int pcpd_get_tuning(pcpd_ctx *ctx, pcpd_tuning *tuning);

/* Options of a context (bit flags). */
typedef enum {
    /* Run the sweeps of pcpd_sweep / pcpd_run in segments of a fixed number of Monte Carlo
     * steps (256 phase launches), each captured into a HIP graph on first use and replayed
     * whenever a segment comes again (same copy parity); the kernels read the substep index
     * from a device clock, so a replay is valid at any starting time. Remainders and density
     * records are launched directly. Ignored while profiling. */
    PCPD_OPT_GRAPH = 1,
    /* Run all phases between two records in one launch of resident workgroups that take work
     * items (phase, tile) in order from an atomic ticket; an item starts once the tiles it
     * reads from have finished the previous phase (per-tile completion flags), so phases
     * overlap and no launch boundary separates them (paper Sec. 3: more independent systems
     * and more tiles than one phase fills). Results are identical. A dependency wait that
     * exceeds its bound (a correct run never does) stops the launch; the next synchronising
     * call returns PCPD_EDEVICE. With PCPD_OPT_GRAPH the persistent launches are captured. */
    PCPD_OPT_PERSISTENT = 2,
    /* Skip the substeps of a tile whose loaded range (interior and halo) holds no particle in
     * any sample: no rule of eq. (1) acts on an empty window, so the tile ends the phase empty
     * and only its zeros are written back. Results are identical; the time of a phase then
     * depends on the state (late-time and extinct runs get cheaper), so rates measured with it
     * are reported apart. */
    PCPD_OPT_SKIP_EMPTY = 4
} pcpd_option;

/* Set the options (an OR of pcpd_option flags; unknown bits: PCPD_EINVAL). A change waits
 * for the context's queued work and drops its captured graphs. */
PCPD_API int pcpd_set_options(pcpd_ctx *ctx, uint32_t options);

/* Pick the kernel shape by timing candidate tiles (blocks per tile x substeps
 * per phase x teams) on this context's own lattice: each trial reads the current
 * copy and writes the spare one, so the state is unchanged. `reps` timed launches
 * per candidate (0 = 3). The choice is cached per process for contexts of the
 * same model, block width and ring sizes, applied to the context and returned
 * in *chosen (may be NULL). Results never depend on the shape.
 * On disk: if the environment variable PCPD_TUNE_CACHE names a file, an entry
 * there for this GPU architecture and key is used without timing (the last
 * matching line wins; an entry written by hand forces a shape), and a shape
 * that had to be timed is appended. A line holds the architecture (e.g.
 * gfx950), model n, B, the number of rings, their total, largest and smallest
 * block counts, then tile columns, substeps per phase and teams. */
PCPD_API int pcpd_autotune(pcpd_ctx *ctx, uint32_t reps, pcpd_tuning *chosen);

/* Timing of the sweep's phase kernels: while enabled, every phase launch is
 * bracketed by a pair of HIP events on the context's stream.
 * pcpd_profile_read synchronises, returns the summed kernel time in
 * milliseconds and the number of launches since the last read, and resets
 * both. Enabling does not change results. */
PCPD_API int pcpd_profile(pcpd_ctx *ctx, int enable);
PCPD_API int pcpd_profile_read(pcpd_ctx *ctx, double *kernel_ms, uint64_t *launches);

/* ---- Allocation-free run ------------------------------------------------
 * For callers that cannot allocate device memory (code that must not call
 * hipMalloc: tight serving loops, harnesses that forbid allocation). The same
 * computation as pcpd_init (start taken from device memory) followed by
 * pcpd_run, with no context: the spare lattice copy, the ring and tile tables,
 * the count records and the device clock live in one fixed workspace that the
 * library holds per GPU (a device variable of about 35 MiB, kept until the
 * process ends). The call allocates nothing, on the device or through any
 * library routine.
 *
 * Limits (PCPD_ELIMIT beyond them, checked before any device work):
 *   planes * sum L           <= PCPD_NOALLOC_MAX_WORDS  (2^22 words, 32 MiB)
 *   n_inst * planes          <= PCPD_NOALLOC_MAX_RINGS
 *   n_times * n_inst * planes <= PCPD_NOALLOC_MAX_RECORDS
 *   (and at most 65536 tiles and 8192 density chunks, which the limits
 *   above imply for B = 64).
 *
 * Arguments: cfg and inst as for pcpd_init, except that inst[i].init and
 * host_words are ignored. dev_lattice: DEVICE memory of the current HIP
 * device, planes * sum L uint64 words laid out as the context keeps them
 * (instance-major, then plane-major, natural site order, 8-byte aligned),
 * holding the lattice at Monte Carlo step t0 on entry and at
 * times[n_times - 1] on return (unchanged if n_times == 0); borrowed for the
 * call. times, n_times, out: as for pcpd_run (times >= t0, strictly
 * increasing; out a host array of n_times * n_inst * planes records).
 * hip_stream: the stream to run on (NULL = null stream), of the current
 * device. Synchronous: returns after the records are on the host.
 * Results are bit-identical to pcpd_init + pcpd_run on the same start.
 * Errors: PCPD_EINVAL / PCPD_EOVERFLOW as pcpd_init and pcpd_run (nothing
 * enqueued), PCPD_ELIMIT, PCPD_EDEVICE for a failed HIP call or kernel.
 * All calls on one GPU share its workspace: calls that overlap in time on
 * the same GPU (two host threads, or streams of one device) race and give
 * undefined results; calls made one after another are independent. */
#define PCPD_NOALLOC_MAX_WORDS (1ull << 22)
#define PCPD_NOALLOC_MAX_RINGS 4096u
#define PCPD_NOALLOC_MAX_RECORDS 65536u
PCPD_API int pcpd_run_noalloc(const pcpd_config *cfg, const pcpd_instance *inst, uint32_t n_inst,
                              uint64_t t0, uint64_t *dev_lattice, const uint64_t *times,
                              uint32_t n_times, pcpd_counts *out, void *hip_stream);

/* Release the context and everything the library allocated for it. */
PCPD_API int pcpd_free(pcpd_ctx *ctx);

/* Description of the HIP failure behind the context's last PCPD_EDEVICE or
 * PCPD_ENOMEM ("none" if there was none); static storage, valid until the
 * library is unloaded. */
PCPD_API const char *pcpd_device_error(pcpd_ctx *ctx);

/* Static description of a status code. */
PCPD_API const char *pcpd_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* PCPD_H */
