/*
 * ec.h -- C ABI of libec: RS(n,p) erasure coding over GF(2^8) executed as
 * compiled XOR straight-line programs (SLPs) on an MI355X (gfx950) GPU.
 *
 * Method: Uezato, "Accelerating XOR-based Erasure Coding using Program
 * Optimization Techniques" (SC'21).  A coding matrix is expanded into a GF(2)
 * bitmatrix (Sec. 1) and turned into an XOR straight-line program (Sec. 2,
 * 4.1), compressed by XorRePair (Sec. 4.3-4.4) and fused into multi-input
 * XORs (Sec. 5.2).  For the GPU the compression runs on column blocks of the
 * bitmatrix (one data block each by default), so that the temporaries a
 * block needs fit in registers, and the program runs in push form: every
 * value (an input strip or a finished temporary) is brought into an
 * accumulator once and XORed into each register slot that consumes it;
 * output rows and open temporaries live in register slots, never in memory.
 * The slot schedule plays the part of the paper's cache pebbling (Sec. 6).
 * A HIP kernel interprets the resulting records over every tile of every
 * strip.
 *
 * Conventions shared by every entry point:
 *  - Status codes only; nothing throws across the ABI.
 *  - Data buffers (device memory) are owned by the caller; programs and
 *    batches are owned by the library and freed with their *_free call,
 *    only after the work queued on them has completed.
 *  - Block layout: each block is one contiguous buffer of S bytes; strip c of
 *    a block is bytes [c*S/8, (c+1)*S/8).  S must be a positive multiple of
 *    128 (so every strip is a whole number of 16-byte lanes) and every block
 *    pointer must be 16-byte aligned (EC_ERR_ALIGN otherwise).
 *  - Symbols: for a byte offset k of the strips and bit b, block i carries
 *    the field element sum_c bit_b(strip_c[k]) x^c; the code is linear over
 *    these symbols (Sec. 1, the byte <-> bit-vector isomorphism).
 *  - Field: GF(2^8) with x^8+x^4+x^3+x^2+1 (0x11D) (Sec. 7.1).
 *  - Launch calls are asynchronous on the given HIP stream (NULL = default
 *    stream); argument errors are reported synchronously, launch failures as
 *    EC_ERR_DEVICE, device faults at the caller's next synchronisation.
 */
#ifndef EC_H
#define EC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ec_program ec_program; /* compiled program: host IR + device bytecode */
typedef struct ec_batch ec_batch;     /* prepared multi-stripe launch */
typedef struct ec_server ec_server;   /* serving loop: streams, events and reusable batches */
typedef struct ihipStream_t *ec_stream; /* a hipStream_t */

typedef enum {
  EC_OK = 0,
  EC_ERR_ARG = 1,               /* bad argument (null pointer, n/p out of range, ...) */
  EC_ERR_ALIGN = 2,             /* block size not a multiple of 128 or pointer not 16-B aligned */
  EC_ERR_TOO_MANY_ERASURES = 3, /* more than p blocks erased */
  EC_ERR_SINGULAR = 4,          /* survivor submatrix of the generator is not invertible */
  EC_ERR_NOMEM = 5,             /* host or device allocation failed */
  EC_ERR_DEVICE = 6,            /* HIP runtime error (no device, launch failure) */
  EC_ERR_UNSUPPORTED = 7,       /* option or size outside what the executor supports */
  EC_ERR_CAPACITY = 8           /* program does not fit the register slot budget; or a
                                   request does not fit a server's budget or arena; or a
                                   batch does not fit ec_batch_run_noalloc's fixed tables */
} ec_status;

/* Optimisation level of a compiled program (the stages of Sec. 7.5). */
enum {
  EC_LEVEL_PLAIN = 0,        /* the plain bitmatrix SLP: every strip XORed into each row it feeds */
  EC_LEVEL_CO = 1,           /* column blocks compressed by XorRePair, binary XORs (Sec. 4.4) */
  EC_LEVEL_CO_FU = 2,        /* compressed then fused (Sec. 5.2) */
  EC_LEVEL_CO_FU_SCHED = 3   /* compressed, fused, strips ordered to keep few temporaries open
                                (the register counterpart of Sec. 6); default */
};

/* Compression algorithm for levels >= EC_LEVEL_CO. */
enum { EC_COMPRESS_XORREPAIR = 0, EC_COMPRESS_REPAIR = 1 };

/* Order in which the executor brings in the input strips (Sec. 6: the
 * schedule of a straight-line program under a bounded cache; here the cache
 * is the register slots).  Temporaries complete as their last source
 * arrives, and the slot schedule is the same for both. */
enum {
  EC_SCHED_PUSH = 0,   /* level EC_LEVEL_CO_FU_SCHED: within each column block, the strip that
                          opens the fewest temporaries net of those it completes next; lower
                          levels: strip order (default) */
  EC_SCHED_GREEDY = 1  /* every level: the order in which the bottom-up greedy heuristic of
                          Sec. 6.6, run on the program's statements for an LRU cache of
                          slot-budget entries, first reads the strips (within each column block
                          from level EC_LEVEL_CO on); the row-split parts take the order the
                          heuristic gives the plain rows */
};

typedef struct {
  uint32_t level;        /* EC_LEVEL_*; default EC_LEVEL_CO_FU_SCHED */
  uint32_t slot_budget;  /* register slots per lane (16 B each); supported: 24, 32, 36, 38, 40,
                            44, 48, 56, 60 (the executor runs 4 waves per SIMD up to 24 slots, 3
                            up to 38, else 2); 0 = default: the first of 24, 32, 38, 44, 48 that
                            holds every output row in one pass over the inputs with a ring of
                            at least 3 strip loads, else the first of 56, 60 that does, else 48
                            (several passes) */
  uint32_t compress;     /* EC_COMPRESS_*; default XorRePair */
  uint32_t block_strips; /* width in strips of the column blocks compressed separately
                            (levels >= CO); 0 = 8, one data block; 8*n = the whole matrix */
  uint32_t prefetch;     /* distance in strips at which strips are touched (4 B per lane)
                            ahead of their register load, so that the load finds them in
                            the L2 cache; 0 = none (NULL opts: the library's default) */
  uint32_t split;        /* EC_SPLIT_*: whether a launch may run the output rows of one
                            tile on different waves (see ec_program_info.n_parts) */
  uint32_t scheduler;    /* EC_SCHED_*; default EC_SCHED_PUSH */
  uint32_t native;       /* EC_NATIVE_* bits: native kernels to compile (below); default 0 */
} ec_compile_opts;

/* Native kernels to compile (ec_compile_opts.native, ec_program_info.native). */
enum {
  EC_NATIVE_WHOLE = 1,  /* the whole program: launches with no row split */
  EC_NATIVE_PAIRS = 2,  /* the pair parts (when the program has them): launches that split into pairs */
  EC_NATIVE_BLOCKS = 4  /* the block parts (when the program has them): launches that split by output block */
};

/* Native kernels (ec_compile_opts.native).  The program's records, a
 * fixed sequence of strip loads, register XORs and strip stores per tile,
 * are also written out as straight-line gfx950 code with every register
 * slot a fixed register group, and compiled at ec_compile_slp time with
 * hiprtc (host only: no device needed; about 1-2 s for an RS(10,4)
 * program).  A single-stripe launch that runs the whole program, one wave
 * per tile (no row split: ec_encode / ec_decode of long stripes), then runs
 * that kernel instead of the interpreter: the same loads, XORs and stores
 * in the same order, with no record dispatch, register indexing or record
 * loads: a fraction of the instructions.  EC_NATIVE_PAIRS compiles the
 * pair parts the same way into one kernel (work item k runs pair part
 * k % n_pair_parts of tile k / n_pair_parts), which then runs every launch
 * that splits into pair parts; it takes about 5 s to compile for RS(10,4).
 * EC_NATIVE_BLOCKS does the same for the block parts (one wave per tile and
 * output block), which then run every launch that splits by output block.
 * With native kernels EC_SPLIT_AUTO takes the native pair parts while
 * there is at most one wave per SIMD (up to 512 KiB blocks for RS(10,4)),
 * then the native block parts while there are at most two (up to 2 MiB),
 * else the native whole program, each only where the program has that
 * kernel, and without them the interpreter's rule (EC_SPLIT_AUTO below).
 * Row and pass splits and batches keep the interpreter.  The kernel is loaded on
 * a device at the program's upload or first launch there and stays loaded
 * until the process ends (identical kernels are loaded once).  Not with
 * EC_SPLIT_STAGED (EC_ERR_UNSUPPORTED); EC_ERR_UNSUPPORTED also if the
 * compiler fails. */

/* Row split.  Unless compiled with EC_SPLIT_NEVER, a program also carries
 * "parts": independent programs that each compute some of the output rows
 * from the inputs they need (scheduled from the plain bitmatrix rows, which
 * make the shortest chains of records, whatever the level), in three sets:
 *  - block parts: up to 8, each a group of whole output blocks (only when
 *    there is more than one output block);
 *  - row parts: up to 32, each one bit row (beyond 4 output blocks, runs
 *    of floor or ceil(8 n_out / 32) consecutive rows);
 *  - pair parts: up to 16, each two consecutive bit rows (beyond 4 output
 *    blocks, runs of floor or ceil(8 n_out / 32) pairs);
 *  - pass parts (only for a program whose rows need several passes over the
 *    inputs): the fewest groups of whole output blocks that each fit one
 *    pass, scheduled from the program itself.  The parts of a tile run on
 *    neighbouring waves of one workgroup at the same time, so each input
 *    strip-tile comes from HBM once and from the caches for the other parts
 *    (a single wave reads it from HBM again on every pass).
 * A launch over a stripe with few tiles then runs one wave per (tile, part)
 * instead of one per tile, which gives short stripes more waves and each
 * wave a shorter chain of records and a deeper load ring, at the cost of
 * reading each input once per part that needs it (mostly from the caches).
 * A batch (ec_batch_*) decides for all its EC_SPLIT_AUTO stripes at once,
 * by the same rule over the work items of the whole batch. */
enum {
  EC_SPLIT_AUTO = 0,   /* the finest set that fits, none if no set does (default): row parts,
                          then pair parts, while one wave per (tile, part) leaves at most two
                          waves per SIMD; block parts while those waves fit in the waves the
                          chip keeps resident for the program's slot budget; else pass parts,
                          when the program has them */
  EC_SPLIT_NEVER = 1,  /* one wave per tile; no parts are built */
  EC_SPLIT_ALWAYS = 2, /* block parts on every launch when the program has them */
  EC_SPLIT_ROWS = 3,   /* row parts on every launch when the program has them */
  EC_SPLIT_PAIRS = 4,  /* pair parts on every launch when the program has them */
  EC_SPLIT_PASSES = 5, /* pass parts on every launch when the program has them */
  EC_SPLIT_STAGED = 6  /* stage parts in LDS (below); only these parts are built */
};

/* Staged launches (EC_SPLIT_STAGED; Sec. 8's multi-level hierarchy and
 * software prefetch, with LDS as the level between the register slots and
 * HBM).  The program carries "stage parts": up to 4 runs of consecutive bit
 * rows, min(4, 8 n_out) of them, as even as can be, each scheduled from the
 * program itself (its level, order and slot budget).  A launch runs one
 * workgroup of 4 waves per tile: the waves copy the tile's 8 n_in input
 * strip-tiles (1 KiB each) into LDS with asynchronous LDS-DMA loads, then
 * wave w runs stage part w with its strip loads served from LDS.  Every
 * input strip-tile is read from HBM once per tile, and a part's slots hold
 * only its own rows.  Needs 8 KiB of LDS per input block: n_in <= 20
 * (EC_ERR_UNSUPPORTED at compile time beyond, or at launch on a device with
 * less LDS per workgroup).  Off by default: measured on RS(10,4), it
 * fetches exactly the algorithmic bytes at every size (the default split of
 * short stripes re-reads inputs across its parts) but, its waves loading
 * nearly every input for a quarter of the rows at 2 waves per SIMD, runs
 * 1.3-2.4x slower than the direct launch from 8 MiB blocks up and within 5%
 * of it at 1 MiB.  A batch runs a staged program whole, one wave per
 * tile. */

typedef struct {
  uint32_t n, p;        /* codec */
  uint32_t n_in;        /* input blocks (n) */
  uint32_t n_out;       /* output blocks (p for encode, number of erasures for decode) */
  uint32_t n_stmt;      /* statements of the optimised SLP */
  uint32_t n_xor2;      /* #xor: sum over statements of (arity - 1) (Sec. 4.1) */
  uint32_t n_mem;       /* #M: sum over statements of (arity + 1) (Sec. 5.1) */
  uint32_t nvar;        /* variables of the optimised SLP (Sec. 4.1; pebbles after Sec. 6.6) */
  uint32_t plain_xor2;  /* #xor of the plain bitmatrix program (ones - rows) */
  uint32_t slots;       /* register slot budget the program was scheduled for */
  uint32_t peak_open;   /* temporaries open at once (slots beside the rows and the ring) */
  uint32_t ring;        /* strip loads in flight ahead of their use */
  uint32_t passes;      /* passes over the inputs per tile (1 unless the rows exceed the slots) */
  uint32_t n_loads;     /* strip loads per tile (inputs used, times passes) */
  uint32_t n_stores;    /* strip stores per tile (= 8 * n_out) */
  uint32_t n_records;   /* executor records per tile */
  uint32_t n_ops;       /* slot XORs per tile (the executor's unit of work) */
  uint32_t n_words;     /* bytecode words */
  uint32_t n_parts;     /* block parts for the row split (0: none, e.g. one output block) */
  uint32_t n_row_parts; /* row parts for the row split (0: none) */
  uint32_t n_pair_parts; /* pair parts for the row split (0: none) */
  uint32_t n_pass_parts; /* pass parts (0: none; the program needs one pass) */
  uint32_t scheduler;   /* EC_SCHED_* the strip order was made with */
  uint32_t n_stage_parts; /* stage parts (EC_SPLIT_STAGED only; 0: none) */
  uint32_t native;      /* EC_NATIVE_* bits of the native kernels the program has */
  const int *in_blocks;  /* n_in block indices (0..n+p-1) read, in argument order */
  const int *out_blocks; /* n_out block indices written, in argument order */
} ec_program_info;

/* Systematic Cauchy generator G = [I_n ; P], P[i][j] = 1/(i + (p + j)) over
 * GF(2^8) (the configured coding matrix; any square submatrix of a Cauchy
 * matrix is nonsingular, as Sec. 1 requires of the decode step).
 * gen: caller buffer of (n+p)*n bytes, row-major.  Needs n >= 1, p >= 0,
 * n + p <= 64.  */
ec_status ec_matrix_cauchy(int n, int p, uint8_t *gen);

/* Generator with parity rows P[r][j] = alpha^(r*j) (alpha = x): the reading
 * of Sec. 7.1 under which the printed XOR counts of the paper's RS(10,4)
 * programs are reproduced.  Same layout and limits as ec_matrix_cauchy. */
ec_status ec_matrix_vandermonde(int n, int p, uint8_t *gen);

/* Compile an XOR program for an encode (n_erased == 0) or for the erasure
 * pattern `erased` (decode).  gen is the (n+p) x n generator (copied).
 * Decode reads the n lowest-indexed surviving blocks and reconstructs every
 * erased block, data or parity (Sec. 1: the surviving rows form M and
 * M^-1 recovers the data).  Needs 1 <= n, 0 <= p, n + p <= 32 (the
 * executor's block table).  Host-only: needs no GPU.  Thread-safe.
 * block_strips must be 0 or 1..8n.
 * Errors: EC_ERR_ARG (also for a duplicate or out-of-range erased index),
 * EC_ERR_TOO_MANY_ERASURES (n_erased > p), EC_ERR_SINGULAR, EC_ERR_CAPACITY,
 * EC_ERR_UNSUPPORTED (level / slot budget not supported), EC_ERR_NOMEM. */
ec_status ec_compile_slp(int n, int p, const uint8_t *gen, const int *erased, int n_erased,
                         const ec_compile_opts *opts /* NULL = defaults */, ec_program **out);

/* Counts and block mapping of a compiled program (Sec. 4.1, 5.1, 6.2
 * measures).  The arrays in *out stay valid until ec_program_free. */
ec_status ec_program_query(const ec_program *prog, ec_program_info *out);

/* Encode (Sec. 1: the codeword is the generator times the data, so the
 * parity blocks are P times the n data blocks, computed here as the
 * program's XORs of bitmatrix rows over the strips): data = n device
 * pointers (blocks 0..n-1), parity = p device pointers (blocks n..n+p-1),
 * each block_bytes long, caller-owned.  prog must be an encode program
 * (EC_ERR_ARG otherwise).  Parity buffers must not overlap each other or any
 * data buffer (EC_ERR_ARG).  Asynchronous on `stream`; EC_ERR_ALIGN,
 * EC_ERR_UNSUPPORTED (strips of 512 MiB or more), EC_ERR_NOMEM / EC_ERR_DEVICE
 * on the program's first upload to the device or a failed launch. */
ec_status ec_encode(const ec_program *prog, const uint8_t *const *data, uint8_t *const *parity,
                    size_t block_bytes, ec_stream stream);

/* Decode (Sec. 1: with M the rows of the generator for n surviving blocks,
 * the data is M^-1 times the survivors, and an erased block e is row e of
 * the generator times that; the program applies these rows, fixed at
 * compile time, to the survivors): survivors = n device pointers in the
 * order info.in_blocks; recovered = n_erased device pointers in the order
 * info.out_blocks, each block_bytes long, caller-owned.  prog must be a
 * decode program (EC_ERR_ARG otherwise); same buffer rules and errors as
 * ec_encode. */
ec_status ec_decode(const ec_program *prog, const uint8_t *const *survivors, uint8_t *const *recovered,
                    size_t block_bytes, ec_stream stream);

/* Copy the program's records to the current device now (synchronously).
 * Otherwise the first launch on a device does it, which a latency-sensitive
 * caller may not want.  Once a program is on the device, ec_encode /
 * ec_decode with it only enqueue one kernel and may be captured into a HIP
 * graph.
 * A program with a native kernel also loads that kernel here.
 * Records live in the device's program pool: device memory taken in chunks
 * of at least 4 MiB (kept until the process ends) and shared by all
 * programs, where identical records are stored once.  ec_program_free drops
 * the program's hold on its records; their space is reused once no program
 * holds them.
 * Errors: EC_ERR_ARG, EC_ERR_NOMEM, EC_ERR_DEVICE. */
ec_status ec_program_upload(ec_program *prog);

/* Copy the records of n programs (each non-null) to the current device: the
 * pool first sets aside, in one piece, the space that all of those not yet
 * there need, so a set of programs takes at most one device allocation
 * (a server's hundreds of erasure patterns, say).  Programs already on the
 * device are skipped.  Synchronous.
 * Errors: EC_ERR_ARG (n < 0, a null pointer), EC_ERR_NOMEM, EC_ERR_DEVICE;
 * on an error the programs before the failing one stay uploaded. */
ec_status ec_program_upload_many(ec_program *const *progs, int n);

/* The source of the program's native kernel `kernel` (EC_NATIVE_WHOLE,
 * EC_NATIVE_PAIRS or EC_NATIVE_BLOCKS; host copy, valid until ec_program_free; *len without a
 * terminating zero, which follows it).  EC_ERR_ARG if the program has no
 * such kernel. */
ec_status ec_program_native_source(const ec_program *prog, int kernel, const char **src, size_t *len);

/* The current device's program pool: chunks of device memory allocated,
 * distinct records held, and bytes of them in use (in 256-byte granules).
 * Any output pointer may be null, not all three (EC_ERR_ARG).
 * EC_ERR_DEVICE if there is no current device. */
ec_status ec_program_pool_stats(int *chunks, int *images, size_t *bytes_used);

void ec_program_free(ec_program *prog);
const char *ec_status_str(ec_status s);

/* ---- inspection (used by tests to check the compiler against the oracle) */

/* Stage of the compilation pipeline to export. */
enum {
  EC_STAGE_PLAIN = 0, /* one statement per bitmatrix row */
  EC_STAGE_CO = 1,    /* after (Xor)RePair */
  EC_STAGE_FU = 2,    /* after XOR fusion */
  EC_STAGE_SCHED = 3, /* after DFS scheduling */
  EC_STAGE_EXEC = 4   /* the program the executor runs, in push form: its temporaries in
                         completion order, then one statement per output row */
};

/* Export one stage as a flat int32 array:
 *   [n_stmt, n_out, { var, arity, op_0 .. op_{arity-1} } * n_stmt, out_0 .. out_{n_out-1}]
 * Terms: t >= 0 is a variable; t == -1 is the zero array; t <= -2 is input
 * strip c = -t - 2 (strip c of input argument c / 8).  Output j*8+r is strip
 * r of output argument j.  *len receives the needed length; nothing is
 * written beyond cap.  Stages PLAIN/CO/FU/SCHED are the paper's whole-matrix
 * pipeline (Secs. 2-6) on this program's bitmatrix, built for inspection;
 * CO/FU/SCHED exist for levels >= CO, FU for >= CO_FU, SCHED for
 * CO_FU_SCHED. */
ec_status ec_program_export(const ec_program *prog, int stage, int32_t *buf, size_t cap, size_t *len);

/* The fused stage (EC_STAGE_FU) scheduled by the bottom-up greedy heuristic
 * of Sec. 6.6 for an abstract LRU cache of `capacity` entries, in the
 * export format above, with pebbles for variables: a statement's var is the
 * pebble its value is put on (pebbles are reused, so a var may be assigned
 * more than once), operands name pebbles or input strips, and the returned
 * terms name the pebbles that hold the outputs at the end.  The DFS
 * heuristic of the same section is EC_STAGE_SCHED.  Needs capacity >= 1 and
 * a program of level >= EC_LEVEL_CO_FU (else EC_ERR_ARG).  Host-only. */
ec_status ec_program_export_greedy(const ec_program *prog, int capacity, int32_t *buf, size_t cap, size_t *len);

/* ---- bandwidth references (not part of the paper's method)
 *
 * Device-to-device copy (non-temporal 16-byte accesses, two per lane per
 * step, 16 workgroups per compute unit): the plain HBM copy ceiling, and the
 * kernel used to calibrate byte counters.  bytes: multiple of 16; both
 * pointers 16-byte aligned (EC_ERR_ALIGN) and not overlapping (EC_ERR_ARG).
 * Asynchronous on `stream`. */
ec_status ec_device_copy(void *dst, const void *src, size_t bytes, ec_stream stream);

/* The data movement of one ec_encode / ec_decode launch without a program:
 * every tile (1 KiB of every strip) reads all n_in input blocks' strips and
 * writes all n_out output blocks' strips, in the executor's tile order, each
 * output strip-tile being the XOR of that tile's n_in * 8 input strip-tiles
 * (a stand-in that needs every input byte).  The ceiling for a coding launch
 * of the same shape.  Same block rules and errors as ec_encode; needs
 * n_in >= 1, n_out >= 0, n_in + n_out <= 32 (EC_ERR_ARG). */
ec_status ec_stripe_stream(const uint8_t *const *in, int n_in, uint8_t *const *out, int n_out, size_t block_bytes,
                           ec_stream stream);

/* The device bytecode the executor runs per tile (host copy). */
ec_status ec_program_bytecode(const ec_program *prog, const uint32_t **words, size_t *n_words);

/* The bytecode of part `part` of a program: block part `part` for
 * 0 <= part < info.n_parts, then row part `part - n_parts` for
 * part < n_parts + n_row_parts, then pair part `part - n_parts -
 * n_row_parts` up to n_parts + n_row_parts + n_pair_parts, then the pass
 * parts up to that plus n_pass_parts, then the stage parts up to that plus
 * n_stage_parts (host copy; same record format as
 * ec_program_bytecode, storing only the part's output rows).  EC_ERR_ARG for
 * a part that does not exist. */
ec_status ec_program_part_bytecode(const ec_program *prog, int part, const uint32_t **words, size_t *n_words);

/* ---- batched execution: many stripes, one persistent launch */

typedef struct {
  const ec_program *prog; /* encode or decode program */
  const uint8_t *const *in;  /* prog's n_in device block pointers */
  uint8_t *const *out;       /* prog's n_out device block pointers */
  size_t block_bytes;        /* multiple of 128 */
} ec_stripe;

/* Prepare a launch over n_stripes stripes: uploads the stripe descriptors
 * and program bytecode to the device (synchronously, on `stream`).  The
 * stripes' buffers and programs must stay valid for every later launch.
 * tile_bytes: bytes per strip one work item covers (a multiple of 1024, the
 * bytes of a strip one wave handles per tile; 0 = 1024).  Programs in one
 * batch must share one slot budget (EC_ERR_UNSUPPORTED otherwise).  The
 * stripes run in no defined order, so every output block must be disjoint
 * from every other output block and from every input block of the batch
 * (EC_ERR_ARG otherwise); input blocks may be shared between stripes. */
ec_status ec_batch_build(const ec_stripe *stripes, int n_stripes, size_t tile_bytes, ec_stream stream,
                         ec_batch **out);

/* Run the batch: one launch of the HIP graph built by ec_batch_build (a
 * one-thread kernel resetting the work counter, then the persistent
 * executor whose waves take chunks of (stripe, tile) work items from that
 * counter).  Launches of one batch must not overlap (they share the
 * counter). */
ec_status ec_batch_launch(ec_batch *batch, ec_stream stream);

/* The same two kernels enqueued directly on `stream` instead of as a graph:
 * for callers that capture their own graphs (no allocation, no memset). */
ec_status ec_batch_enqueue(ec_batch *batch, ec_stream stream);

/* A reusable batch for serving loops: ec_batch_create allocates an empty
 * batch; ec_batch_set fills it for a new set of stripes, staging the tables
 * in pinned host memory and enqueueing their copies on `stream` without
 * waiting (device buffers grow when needed and are never freed before
 * ec_batch_free).  The previous launch of the batch must have completed
 * before ec_batch_set is called again.  Run it with ec_batch_enqueue on the
 * same stream.  Same argument rules and errors as ec_batch_build. */
ec_status ec_batch_create(ec_batch **out);
ec_status ec_batch_set(ec_batch *batch, const ec_stripe *stripes, int n_stripes, size_t tile_bytes,
                       ec_stream stream);

/* Size the batch's tables now for up to n_stripes stripes and n_items work
 * items, so that later ec_batch_set calls up to those sizes allocate
 * nothing (allocation and release can synchronise the device).
 * Errors: EC_ERR_ARG, EC_ERR_DEVICE (other current device), EC_ERR_NOMEM. */
ec_status ec_batch_reserve(ec_batch *batch, int n_stripes, size_t n_items);

/* Number of work items and total input/output bytes of a batch. */
ec_status ec_batch_query(const ec_batch *batch, size_t *n_items, size_t *in_bytes, size_t *out_bytes);

void ec_batch_free(ec_batch *batch);

/* ---- for callers that cannot allocate
 *
 * For code that must not allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one batched
 * launch over `stripes`, as ec_batch_set + ec_batch_enqueue on `stream`,
 * whose work counter, stripe descriptors and work items live in a fixed
 * device array of EC_NOALLOC_SCRATCH_BYTES per device (part of the library,
 * held by each device it runs on until the process ends) instead of memory
 * the library allocates.  The call allocates nothing, on the device or the
 * host: it fills the tables in a static host array, copies them into the
 * device array with hipMemcpyAsync on `stream` and launches.
 *  - Every call on one device shares that device's array: calls on the same
 *    stream run in order, but calls whose launches overlap on one device
 *    (different streams, or threads racing to different streams) race on
 *    the array and give undefined results.  Host threads are serialised
 *    inside the call.
 *  - Every program must already be on the current device (ec_program_upload
 *    or an earlier launch with it): a program that is not gives EC_ERR_ARG,
 *    since uploading it would allocate.
 *  - At most EC_NOALLOC_MAX_STRIPES stripes, and work items (one per
 *    tile_bytes of a strip, times the parts of the batch's row split) within
 *    what the array holds after the descriptors (997,312):
 *    EC_ERR_CAPACITY otherwise.
 *  - Otherwise the same arguments, rules and errors as ec_batch_set
 *    (outputs disjoint from each other and from every input).  Results are
 *    those of ec_batch_build / ec_batch_launch on the same stripes. */
#define EC_NOALLOC_SCRATCH_BYTES (8u << 20)
#define EC_NOALLOC_MAX_STRIPES 1024
ec_status ec_batch_run_noalloc(const ec_stripe *stripes, int n_stripes, size_t tile_bytes, ec_stream stream);

/* ---- serving: a request loop with continuous batching
 *
 * Not part of the paper's method (which codes one stripe at a time): the
 * loop that serves a stream of independent encode and decode requests with
 * the programs above.  ec_server_run admits arrived requests, in arrival
 * order, while their input + output bytes fit budget_bytes (counting every
 * request in flight) and their outputs fit a first-fit arena in the
 * caller's device buffer; spreads the arrived requests' work (their bytes
 * read and written) evenly over the free slots and packs each slot's share
 * (in arrival order, at least one request and at most max_batch, of one
 * slot budget) into one launch on that slot's stream, a plain
 * ec_encode / ec_decode launch for one request and a reusable ec_batch for
 * more; and keeps admitting while earlier launches run, so requests
 * admitted meanwhile overlap with them on the device.  Completion is found
 * by polling each busy slot's event, on the caller's thread, without
 * sleeping (the loop holds one host core while it runs). */

typedef struct {
  double arrival_s;          /* arrival, seconds after the run starts; nondecreasing over a run */
  const ec_program *prog;    /* encode or decode program */
  const uint8_t *const *in;  /* prog's n_in device input pointers (info.in_blocks order), 16-byte
                                aligned and outside the arena (checked up front) */
  size_t block_bytes;        /* multiple of 128 */
} ec_request;

typedef struct {
  size_t budget_bytes; /* admission limit on the input + output bytes of requests in flight */
  int n_slots;         /* launches in flight, one stream each: 1..16 */
  int max_batch;       /* requests per launch: >= 1 */
} ec_serve_opts;

/* Called on the loop's thread when a launch has completed, before its
 * requests' output space is reused: the requests' indices in the run's
 * array and the byte offsets of their outputs in the arena (output j of a
 * request with block_bytes b at offset + j * b). */
typedef void (*ec_serve_done_fn)(void *user, const int *ids, int n_ids, const size_t *out_off);

/* A server over the caller's device arena (16-byte aligned, at least 4 KiB;
 * it must outlive the server) on the current device: creates n_slots
 * streams (default priority, non-blocking), their events and batches.
 * Errors: EC_ERR_ARG, EC_ERR_ALIGN, EC_ERR_NOMEM, EC_ERR_DEVICE. */
ec_status ec_server_create(uint8_t *arena, size_t arena_bytes, const ec_serve_opts *opts, ec_server **out);

/* Serve n_reqs requests to completion.  Before the clock starts, every
 * program is copied to the device, the batches' tables are sized, and each
 * slot budget's kernels run once on every stream (tiny launches on the
 * arena's first bytes).  realtime = 1: request i is admitted no earlier
 * than arrival_s after the start; 0: every request is present at once.
 * done_s[i] receives request i's completion time on the same clock (when
 * its slot's event was seen complete); out_offsets[i] the arena offset its
 * outputs were placed at (the bytes stay there until a later request takes
 * the space, or a later run's warm-up of a new slot budget writes the
 * arena's first 4 KiB); *wall_s the run's length and *n_batches the
 * launches made (out_offsets, wall_s and n_batches may be NULL).  Checked up front:
 * arrival order, sizes and input alignment (EC_ERR_ALIGN), inputs outside
 * the arena (EC_ERR_ARG), and that every request fits the budget and the
 * arena alone (EC_ERR_CAPACITY).  On a launch or device
 * error the loop waits for the work in flight and returns the error.  One
 * thread at a time per server. */
ec_status ec_server_run(ec_server *server, const ec_request *reqs, int n_reqs, int realtime,
                        ec_serve_done_fn on_done, void *user, double *done_s, size_t *out_offsets, double *wall_s,
                        int *n_batches);

/* Waits for the server's streams, then releases them, the events and the
 * batches (not the arena). */
void ec_server_free(ec_server *server);

#ifdef __cplusplus
}
#endif
#endif /* EC_H */
