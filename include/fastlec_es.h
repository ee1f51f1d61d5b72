/*
 * fastlec_es.h - exact simulation (ES) of And-Inverter-Graph miters on AMD
 * Instinct MI355X (gfx950).  C ABI; plain pointers and sizes only.
 *
 * What is computed.  A circuit is a latch-free AIG (paper, Section 2.1).  It
 * is read as a miter: its miter value at an input assignment is the OR of all
 * of its outputs, and the circuit is EQUIVALENT iff that value is 0 for every
 * assignment (paper, Section 2.1: XOR paired outputs, OR the results,
 * equivalent iff the miter output is identically zero).  Exact simulation
 * enumerates every assignment of the n primary inputs and checks the miter
 * output (paper, Section 2.2, "Exact Simulation"); the result is either
 * EQUIVALENT or the counterexample with the lowest index.
 *
 * Patterns.  Pattern p in [0, 2^n) assigns bit i of p to primary input i (the
 * i-th input of the AIGER file).  A "word" is 64 consecutive patterns:
 * word w holds patterns 64w .. 64w+63.  The space has W = max(1, 2^(n-6))
 * words; for n < 6 word 0 holds every pattern.  n must be at most 63.
 *
 * Errors.  Every int-returning function returns FASTLEC_OK (0) or a negative
 * status.  No C++ exception crosses this boundary.  fastlec_es_last_error()
 * returns a message for the last failing call on the calling thread.
 *
 * Threads and streams.  A circuit handle is immutable after loading; several
 * threads may check the same handle at once, on the same or different streams.
 * Calls block the calling host thread until their results are on the host.
 */
#ifndef FASTLEC_ES_H
#define FASTLEC_ES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
enum {
    FASTLEC_OK = 0,
    FASTLEC_ERR_PARSE = -1,        /* malformed AIGER (bad header, literal, cycle, undefined variable) */
    FASTLEC_ERR_UNSUPPORTED = -2,  /* latches or other sequential sections, or more than 63 inputs */
    FASTLEC_ERR_NOMEM = -3,        /* host or device allocation failed */
    FASTLEC_ERR_DEVICE = -4,       /* HIP runtime or hipRTC failure, or no usable gfx950 device */
    FASTLEC_ERR_INVALID = -5,      /* bad argument (null pointer, empty range, unknown option value) */
    FASTLEC_CANCELLED = -6,        /* the cancel flag was raised; result carries progress */
    FASTLEC_TIMEOUT = -7,          /* the deadline passed; result carries progress */
    FASTLEC_REJECTED = -8          /* server: the job can never fit the memory budget */
};

/* ---- verdicts ------------------------------------------------------------ */
enum { FASTLEC_EQUIVALENT = 0, FASTLEC_NONEQUIVALENT = 1 };

/* ---- kernels ------------------------------------------------------------- */
enum {
    FASTLEC_KERNEL_AUTO = 0,        /* specialized for large spaces, interpreter otherwise */
    FASTLEC_KERNEL_INTERP = 1,      /* generic interpreter, node values in LDS */
    FASTLEC_KERNEL_SPECIALIZED = 2, /* straight-line kernel compiled for this circuit, values in VGPRs */
    FASTLEC_KERNEL_INTERP_HBM = 3   /* generic interpreter, node values in device memory */
};

typedef struct fastlec_es_circuit fastlec_es_circuit; /* opaque, immutable after load */

typedef struct {
    uint32_t num_pis;          /* n */
    uint32_t num_ands;         /* AND gates in the file */
    uint32_t num_ands_tfi;     /* AND gates in the fan-in cone of the outputs (N) */
    uint32_t num_outputs;
    uint32_t peak_live_slots;  /* S: node values alive at once under the planned order */
    uint32_t num_instrs;       /* interpreter instructions (N plus output-only instructions) */
    uint32_t levels;           /* logic depth of the cone */
    uint32_t num_xors;         /* three-AND XORs (x&y, ~x&~y, ~t1&~t2, inner gates read once) that the
                                  interpreter's bundled streams run as one XOR instruction each */
    uint32_t interp_rows;      /* value-file rows of the interpreter's stream in bundles of 4 (constant,
                                  inputs, slots, sink): up to 232 rows live in VGPRs (register tier) */
} fastlec_es_info;

typedef struct {
    int device;                /* HIP device ordinal */
    void *hip_stream;          /* hipStream_t to run on; NULL = the library's stream for the device */
    uint32_t words_per_thread; /* interpreter: 32-bit pattern words per lane per slot (1, 2, 4); 0 = tuned */
    uint32_t tile_words;       /* 64-pattern words claimed per work unit; 0 = tuned */
    uint32_t wg_size;          /* threads per workgroup (64..1024, multiple of 64); 0 = tuned */
    int kernel;                /* FASTLEC_KERNEL_* */
    uint64_t begin_word;       /* check words [begin_word, end_word); 0,0 = the whole space */
    uint64_t end_word;
    double deadline_s;         /* > 0: stop with FASTLEC_TIMEOUT after this many seconds */
    volatile int *cancel_flag; /* host memory; nonzero = stop with FASTLEC_CANCELLED; may be NULL */
    void *dev_scratch;         /* fastlec_es_check only, optional: caller-owned device memory on `device`
                                  (256-byte aligned, dev_scratch_bytes long, e.g. a torch tensor) that
                                  holds the launch's control block (claim counters, best value,
                                  descriptor) and, on the device-memory interpreter tier, its value
                                  files, instead of the library's buffers; written in the call's
                                  stream order, free again when the call returns.  Too small or
                                  misaligned: FASTLEC_ERR_INVALID naming the bytes needed.  Batches,
                                  servers, simulation and fastlec_es_check_noalloc ignore it. */
    size_t dev_scratch_bytes;
} fastlec_es_options;

typedef struct {
    int32_t verdict;             /* FASTLEC_EQUIVALENT / FASTLEC_NONEQUIVALENT; a negative status on a
                                    check stopped by its deadline or cancel flag, or a failed server job */
    uint32_t reserved;
    uint64_t cex;                /* lowest failing pattern in the range; valid iff NONEQUIVALENT */
    uint64_t patterns_evaluated; /* patterns whose miter value the answer establishes: the whole range when
                                    EQUIVALENT (2^n for a full check), range start .. cex when not */
    uint64_t next_word;          /* resume point: first word not known to be clean */
    double plan_ms;              /* host planning time (at load) */
    double compile_ms;           /* specialized-kernel compile time paid by this call (0 if cached) */
    double kernel_ms;            /* device time of the simulation kernel(s) */
    double queued_ms;            /* server: admission - submission (host steady clock); 0 otherwise */
    double latency_ms;           /* server: completion - submission (host steady clock); 0 otherwise */
    double predicted_ms;         /* the runtime model's prediction (fastlec_es_predict): plain and batched
                                    checks, the kernel time on the kernel that ran; server, the ETA at
                                    admission = the job's interpreter time alone x the jobs in flight then */
} fastlec_es_result;

/* Fill *opts with defaults: device 0, library stream, tuned schedule, whole space. */
void fastlec_es_options_init(fastlec_es_options *opts);

/* Load an AIGER file from memory (ASCII "aag" or binary "aig", detected from the header),
 * validate it (no latches, n <= 63, topologically orderable), extract the output cone and
 * plan it (evaluation order, reference-count slot map, instruction stream; paper,
 * Section 3.3 "Instructionalized ES").  bytes: host memory, len bytes, caller-owned, not
 * retained.  *out receives a handle owned by the caller until fastlec_es_free. */
int fastlec_es_load_aig(const void *bytes, size_t len, fastlec_es_circuit **out);

/* As fastlec_es_load_aig, reading the file at path. */
int fastlec_es_load_aig_file(const char *path, fastlec_es_circuit **out);

/* Sizes of a loaded circuit. */
int fastlec_es_info_get(const fastlec_es_circuit *c, fastlec_es_info *info);

/* Exact simulation of one circuit over the option's word range (paper, Section 2.2 and
 * Section 3.3).  opts may be NULL (defaults).  Blocks until *out is filled. */
int fastlec_es_check(const fastlec_es_circuit *c, const fastlec_es_options *opts, fastlec_es_result *out);

/* Exact simulation of k circuits of different sizes and input counts (whole space each; the
 * option's word range is ignored).  With kernel AUTO, circuits that the runtime model
 * (fastlec_es_predict) gives to the specialized kernel are compiled together (up to 64 kernels
 * per hipRTC program) and run as their own launches (kernel_ms their own, compile_ms their
 * share of their program's compile); a circuit whose kernel does not compile runs on the
 * interpreter instead.  With kernel SPECIALIZED every circuit runs on its specialized kernel
 * that way.  Of the others, those predicted to take at least 1 ms on the interpreter run as
 * their own launches with their own schedule (unless the options fix words_per_thread or
 * wg_size); the rest are grouped by value-file size (the register tier's 104, 144 and 232 rows,
 * above that powers of two of the row count); each group
 * is one persistent interpreter launch over all its cones, in longest-processing-time order by
 * the runtime model's time, with a tuned schedule (or the option's schedule fields) and recorded
 * once as a hipGraph; their kernel_ms is the sum over the groups.  cs: k handles; out: k
 * results.  An entry's own error (a null handle) is reported in that entry: its verdict is the
 * negative status (FASTLEC_ERR_INVALID) and its other fields are zero; the other entries are
 * checked and valid, and the call returns the first entry's status.  A device or runtime failure
 * fails the whole call with its status; the out entries are then not valid. */
int fastlec_es_check_batch(const fastlec_es_circuit *const *cs, size_t k, const fastlec_es_options *opts,
                           fastlec_es_result *out);

/* ---- exact simulation without device allocation --------------------------- */

/* Bytes of the library's static device array used by fastlec_es_check_noalloc (one per
 * device the library runs on, held until the process ends). */
#define FASTLEC_NOALLOC_SCRATCH_BYTES (1u << 20)

/* For callers that cannot allocate device memory (code that must not call hipMalloc, such as
 * work recorded under HIP graph capture, tight serving loops, harnesses that forbid it): the
 * same check as fastlec_es_check with the interpreter kernel and value files in registers or
 * LDS, whose control block, best value, descriptor and a copy of the circuit's instruction
 * stream live in a static device array of FASTLEC_NOALLOC_SCRATCH_BYTES bytes instead of
 * library allocations.  It calls no hipMalloc, hipFree, hipHostMalloc or event creation; it copies
 * from pageable host memory and waits on the stream.  The first library call on a device
 * (any entry point) sets the device up (properties, library streams, the array's address);
 * make that call outside any code that must not allocate.
 * opts: device, hip_stream, words_per_thread, wg_size, tile_words and the word range as in
 * fastlec_es_check; kernel must be AUTO or INTERP; deadline and cancel flag must be unset.
 * Same answer fields as fastlec_es_check; kernel_ms is the host time from the first upload to
 * the end of the wait (no HIP events are created).
 * Errors: FASTLEC_ERR_INVALID when the bundled instruction stream does not fit the array
 * (about 37,000 instructions at 28 bytes each when the value file fits in registers, about
 * 65,000 at 16 bytes in LDS), when the circuit's value file fits in neither, or for the
 * options above.  The array keeps the last call's contents; every call uploads all of it that
 * it reads.  Calls on one device share the array: the library lets one run at a time per
 * device (a host lock held until the call's results are on the host); calls that overlap on
 * one device from outside this library's lock (another copy of the library in the process)
 * would race. */
int fastlec_es_check_noalloc(const fastlec_es_circuit *c, const fastlec_es_options *opts, fastlec_es_result *out);

/* Release a handle (NULL is allowed). */
void fastlec_es_free(fastlec_es_circuit *c);

/* Message of the last failing call on this thread ("" if none). */
const char *fastlec_es_last_error(void);

/* ---- serving: continuous batching ---------------------------------------- */
typedef struct fastlec_es_server fastlec_es_server;

typedef struct {
    uint64_t submitted, completed, rejected, steps;
    uint64_t active, queued;             /* jobs in flight / waiting now */
    uint64_t charge_in_use_bytes, budget_bytes, peak_charge_bytes;
    uint64_t device_bytes;               /* device memory the server actually holds (tables, value files) */
    uint64_t max_active;                 /* most jobs in flight at once so far */
    double busy_ms;                      /* summed device time of the step kernels */
    uint64_t specialized_slices;         /* job slices run on a job's specialized kernel */
} fastlec_es_server_stats;

/* Start a serving loop on opts->device (continuous batching).  Submitted jobs wait in a
 * queue until admitted; a job is admitted when its charge fits beside the charges of the
 * jobs in flight: charge = peak_live_slots * min(W, chunk_words) * 8 bytes, the node-value
 * slots of its 64-pattern words in flight (W = 2^(n-6) words; chunk_words = 2^22 unless the
 * environment sets FASTLEC_ES_SERVER_CHUNK_WORDS).  The charge is a model of the memory a job
 * would hold with its values materialised; the device memory the server really holds (its job
 * table, about 2.3 MB, plus the value files of jobs too large for LDS, whose launch grid is
 * capped to fit) is kept within budget_bytes too and reported as device_bytes.
 * FASTLEC_ERR_INVALID if budget_bytes does not exceed the job table.  Every step is one interpreter launch
 * over the next slice of every job in flight, so jobs that arrive while others run share
 * the device with them; a job retires as soon as its answer is final (all patterns clean,
 * or the lowest failing pattern known).  Job descriptors and best-so-far values stay in a
 * device-resident job table between steps.  A job whose remaining interpreter time is
 * estimated well above the time to compile its specialized kernel is compiled on a
 * background thread meanwhile (one thread per compile helper process, each compiling one job's
 * kernel in a helper; without the helper program one thread compiling up to eight jobs' kernels
 * as one program); its later slices run on that kernel (same ascending slices, same answer).
 * FASTLEC_ES_SERVER_JIT=0 turns this off.  Slices are sized for steps of
 * FASTLEC_ES_SERVER_STEP_MS (default 10) ms from a running rate estimate that starts at
 * FASTLEC_ES_SERVER_RATE node*patterns/s (default 1e14).  opts: device, stream, schedule
 * fields; the word range, deadline and cancel fields are ignored.  budget_bytes > 0. */
int fastlec_es_server_create(const fastlec_es_options *opts, size_t budget_bytes, fastlec_es_server **out);

/* Queue a job; never blocks.  The circuit must stay alive until the job is polled done.
 * FASTLEC_REJECTED if its charge exceeds the whole budget. */
int fastlec_es_server_submit(fastlec_es_server *s, const fastlec_es_circuit *c, uint64_t *ticket);

/* 1 and *out filled when the job is done, 0 when not yet (wait = 0), or a negative status.
 * wait != 0 blocks until done. */
int fastlec_es_server_poll(fastlec_es_server *s, uint64_t ticket, fastlec_es_result *out, int wait);

/* Counters since creation. */
int fastlec_es_server_stats_get(fastlec_es_server *s, fastlec_es_server_stats *st);

/* Stop the server thread and free its memory; pending jobs are dropped. */
void fastlec_es_server_destroy(fastlec_es_server *s);

/* ---- random-pattern simulation (candidate equivalences for sweeping) ------- */

/* Logic simulation that opens a sweeping flow: simulate the circuit on given input words
 * and find potentially equivalent (PE) nodes (paper, Section 2.3, step 1; its stability
 * and entropy features, Section 3.2, come from the same simulation).
 *
 * fastlec_es_simulate: the value of every variable of c on num_words columns of input words.
 *   pi_words  device pointer, n rows of num_words 32-bit words, row-major (row i = input i;
 *             bit j of word k = the input's value in simulated pattern 32k + j).  Caller-owned,
 *             read only.  May be NULL when n = 0.
 *   sig       device pointer, (max_var + 1) rows of num_words words, row-major, caller-owned,
 *             written completely: row 0 = constant false, rows 1..n = the input words, row
 *             n+1+k = AND gate k of the file (variables renumbered as in the loaded circuit:
 *             the file's own numbering when its inputs are variables 1..n and its AND gates
 *             n+1..M in order).  Every AND gate is simulated, also gates outside the outputs'
 *             cone.  max_var = num_pis + num_ands (fastlec_es_info).
 *   opts      device, stream, words_per_thread (default 1; 4 uses 8-gate bundles, else 16),
 *             wg_size and kernel (FASTLEC_KERNEL_INTERP_HBM forces value files in device memory)
 *             are honoured; may be NULL.
 *   kernel_ms if not NULL, the kernel's time (HIP events on the launch stream).
 * Runs on the option's stream (or the library's own stream): the caller's device buffers must
 * be ready in that stream's order, so pass the stream that produced them (e.g. torch's current
 * stream for tensors torch just filled).  Blocks until sig is written.  FASTLEC_ERR_INVALID for
 * null pointers or num_words = 0.
 *
 * fastlec_es_signature_hash: per row r of a signature matrix (device, rows x num_words,
 *   row-major): ones[r] = number of 1 bits; hash[r] = sum over words k of
 *   word'_k * (fmix32(k mod 2^32) | 1) mod 2^64, where word' is the row complemented when
 *   bit 0 of its word 0 is 1 (so a node and its complement hash alike) and fmix32 is the
 *   MurmurHash3 32-bit finaliser.  hash and ones: device pointers, rows entries each,
 *   caller-owned.  Same stream rule as fastlec_es_simulate.  Blocks until written.
 *
 * fastlec_es_classes: host arrays.  class_of[r] = the lowest row whose hash equals hash[r]
 *   (the class representative; a row is PE with its representative, with complement
 *   iff their rows differ in bit 0 of word 0). */
int fastlec_es_simulate(const fastlec_es_circuit *c, const uint32_t *pi_words, uint64_t num_words, uint32_t *sig,
                        const fastlec_es_options *opts, double *kernel_ms);
int fastlec_es_signature_hash(const uint32_t *sig, uint64_t rows, uint64_t num_words, uint64_t *hash, uint64_t *ones,
                              const fastlec_es_options *opts, double *kernel_ms);
int fastlec_es_classes(const uint64_t *hash, uint64_t rows, uint32_t *class_of);

/* ---- sub-miters by virtual sweeping (host only) ----------------------------- */

/* The paper's scheduling units: imitate one sweeping pass without proving anything.  Each
 * candidate pair keeps only the fan-in cones of its two nodes, and every earlier candidate is
 * merged into its class representative as if already proven (paper, Section 3.2, data
 * features preparation; the sweeping flow of Section 2.3).
 *
 * class_of  host, rows = max_var + 1 entries: representative of each variable (the lowest
 *           member of its class, class_of[u] <= u), as fastlec_es_classes returns.
 * polarity  host, rows entries: bit 0 of word 0 of each variable's signature row (its value
 *           at the first simulated pattern).  u and class_of[u] are candidates for equality
 *           when their polarities agree and for complement when they differ.
 * target    an AND variable with class_of[target] < target.
 * Rules: a literal 2u + c of a non-representative AND u is read as 2 class_of[u] +
 * (c ^ polarity[u] ^ polarity[class_of[u]]); target's own gate is kept with its fan-ins read
 * so; the kept gates are those reachable from target's read fan-ins and from its
 * representative r; the output is XOR(target, r ^ (polarity[target] ^ polarity[r])), as
 * three AND gates t1 = a & b, t2 = ~a & ~b, out = ~t1 & ~t2.  It is constant 0 iff the
 * pair is equivalent under the merges.
 * Text: ASCII AIGER, no symbols.  Inputs = the original inputs in the support, ascending,
 * as variables 1..k; then the kept gates in ascending original order (operands in the
 * original order); then t1, t2, out.
 * buf/len   the text, NUL-terminated; *needed (may be NULL) = bytes it needs with the NUL.
 *           buf may be NULL to ask for the size; a short buf gets FASTLEC_ERR_INVALID.
 * inputs    may be NULL; else at least num_pis entries: original index of each sub-miter
 *           input.  *num_inputs (may be NULL) = k.
 * FASTLEC_ERR_INVALID for a wrong rows count, a target that is not a non-representative
 * AND, a representative above its member, or a polarity entry other than 0 and 1. */
int fastlec_es_submiter_aag(const fastlec_es_circuit *c, const uint32_t *class_of, const uint8_t *polarity,
                            uint64_t rows, uint32_t target, char *buf, size_t len, size_t *needed,
                            uint32_t *inputs, uint32_t *num_inputs);

/* ---- runtime model (host only) -------------------------------------------- */

/* Predicted kernel times of a plain check of c over [begin_word, end_word) (0, 0 = the whole
 * space), by the paper's runtime form (linear in gates, exponential in inputs; Section 3.2,
 * runtime prediction) fitted per kernel on MI355X with a fixed launch cost:
 *   interp_ms       t0 + N * max(patterns / R, L); N = gate instructions of the bundled stream
 *                   (num_instrs - 2 * num_xors); R depends on the value-file size (S)
 *   specialized_ms  t0 + (LUT steps) * max(1, patterns / 2048) / R
 *   compile_ms      hipRTC compile of the specialized kernel: c0 + c1 * (LUT steps)
 * Median errors on the fitting set: 6%, 15%, 0.7%.  Outputs may be NULL; asking for
 * specialized_ms or compile_ms builds the circuit's LUT program (host time).  The AUTO kernel
 * choice of fastlec_es_check uses the same model. */
int fastlec_es_predict(const fastlec_es_circuit *c, uint64_t begin_word, uint64_t end_word, double *interp_ms,
                       double *specialized_ms, double *compile_ms);

/* ---- memory held by the library -------------------------------------------- */

/* Bytes of device memory and of pinned host memory that the library's buffer pool holds on a
 * device (in use or free for reuse), since the process started.  Per-circuit instruction
 * streams, server tables, compiled kernels and the no-allocation array are not counted.
 * Outputs may be NULL. */
int fastlec_es_memory_get(int device, uint64_t *device_bytes, uint64_t *pinned_bytes);

/* ---- roofline probe -------------------------------------------------------- */

/* Issue rate of gfx950's integer VALU for the instructions the specialized kernel is made of:
 * 16 independent chains (a result is read 16 instructions after it is written), 256
 * instructions per loop iteration, waves_per_simd (1..8) waves per SIMD on every CU, iters
 * (>= 1) iterations per wave.  variant 0: v_bitop3_b32 (a three-input LUT) with three VGPR
 * sources in three different register banks; 1: v_bitop3_b32 with two VGPR sources and one
 * SGPR; 2: v_xor_b32.  *instr_per_s = wave64 VALU instructions per second of the loop,
 * *kernel_ms = kernel time (HIP events, the library's stream).  Outputs may be NULL.  This is
 * the measured side of the specialized kernel's roofline (the published figure being 256 CUs x
 * 128 lanes x 2.4 GHz, two wave64 instructions per CU per clock). */
int fastlec_es_valu_probe(int device, uint32_t variant, uint32_t waves_per_simd, uint32_t iters,
                          double *instr_per_s, double *kernel_ms);

/* ---- diagnostics (no GPU needed) ------------------------------------------ */

/* Compile the specialized kernel of c for gfx950 with hipRTC (cached per circuit and by
 * source hash) without running it.  waves_per_eu: occupancy target 1..8.  Outputs may be
 * NULL: *compile_ms = compile time paid by this call (0 when cached), *code_bytes = size of
 * the code object. */
int fastlec_es_compile_specialized(const fastlec_es_circuit *c, int waves_per_eu, double *compile_ms,
                                   size_t *code_bytes);

/* Compile the specialized kernels of k circuits together as hipRTC programs of up to 64 kernels
 * each (every kernel under its own entry point), without running them; no GPU needed.  Kernels
 * already compiled or cached are reused.  hipRTC's fixed cost (about 0.1 s per program) is paid
 * once per program instead of once per circuit.  With at least 24 kernels to compile they are
 * split into several programs of at least 12 kernels, compiled FASTLEC_ES_RTC_PROCS at a time
 * (default min(8, half the host threads)) by child processes running the helper program
 * fastlec_es_rtc, which sits beside the library; a program whose helper fails, is missing or runs
 * longer than FASTLEC_ES_RTC_TIMEOUT_S seconds (300) is compiled in this process.  Helpers start
 * with only stdin, stdout and stderr open and are always waited for before the call returns.  *compile_ms (may be NULL) = total compile time paid by this call.  Later checks of
 * these circuits use the kernels. */
int fastlec_es_compile_specialized_many(const fastlec_es_circuit *const *cs, size_t k, int waves_per_eu,
                                        double *compile_ms);

/* Copy the specialized kernel's HIP source into buf (len bytes, NUL-terminated, truncated
 * to fit) and return the length it needs including the NUL.  buf may be NULL. */
size_t fastlec_es_specialized_source(const fastlec_es_circuit *c, int waves_per_eu, char *buf, size_t len);

/* Replay the interpreter instruction stream planned with `bundle` (1, 4, 8 or 16) on the host,
 * with the kernels' bundle semantics, for the 32-pattern half-words hw .. hw+count-1
 * (half-word h holds patterns 32h .. 32h+31, bit j = pattern 32h+j).  out: count host
 * words of miter values.  Checks the plan's slot map first (FASTLEC_ERR_INVALID if broken).
 * bundle 0 replays the register tier's encoded stream (bundles of 4 with precomputed masks,
 * rows taken from the low 8 bits of each word, outputs only in marked bundles), as that
 * kernel reads it; FASTLEC_ERR_INVALID when the value file does not fit that tier. */
int fastlec_es_host_replay(const fastlec_es_circuit *c, uint32_t bundle, uint64_t hw, uint64_t count,
                           uint32_t *out);

/* Evaluate the specialized kernel's program (the cone mapped onto three-input LUTs, scalar
 * steps and plan-time constant words) on the host for half-words hw .. hw+count-1, into
 * out (count host words of miter values). */
int fastlec_es_host_replay_specialized(const fastlec_es_circuit *c, uint64_t hw, uint64_t count, uint32_t *out);

#ifdef __cplusplus
}
#endif
#endif /* FASTLEC_ES_H */
