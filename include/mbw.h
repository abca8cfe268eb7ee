/*
 * mbw — batched (l,c)-SMEM seeding with sampled-SA locate on one MI355X (gfx950) GPU.
 *
 * Plain C ABI: opaque handles, plain pointers and sizes, integer status codes.  No call throws
 * or aborts; every entry point returns MBW_OK (0) or a negative MBW_E_* code, and
 * mbw_last_error() gives a message for the calling thread's last failure.
 *
 * Paper: "Fast genomic read alignment with minibwa" (arXiv 2606.15357).  Notation follows its
 * Section 2.1: R is the reference, T = R . revcomp(R) . $ with n = |T|, S the suffix array,
 * B the BWT, pi(a,k) the LF-mapping, and (k, k', s) = (lo(P), lo(revcomp P), occ(P)) the
 * double-strand SA interval ("ds-interval") of a string P.
 */
#ifndef MBW_H
#define MBW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------------------------ */
#define MBW_OK          0
#define MBW_E_INVAL    -1   /* bad argument (sizes, ranges, NULL handle)                          */
#define MBW_E_NOMEM    -2   /* device or host allocation failed                                   */
#define MBW_E_HIP      -3   /* a HIP runtime call failed (message names it)                       */
#define MBW_E_IO       -4   /* file could not be opened, read or written                          */
#define MBW_E_FORMAT   -5   /* index file has a bad magic, version, size or checksum              */
#define MBW_E_CAPACITY -6   /* a caller-provided buffer is too small (required sizes reported)     */
#define MBW_E_BUSY     -7   /* serving: queue full on submit, or request not finished on wait      */

const char *mbw_strerror(int code);
/* Message of the calling thread's last failed call ("" if none).  Valid until the next call. */
const char *mbw_last_error(void);

/* ---- index -------------------------------------------------------------------------------- */
typedef struct mbw_index mbw_index;

typedef struct {
  int sa_sample;        /* r: S(x) is kept for rows x that are multiples of r (Section 2.4);
                           1 <= r <= 1024.  Locate walks take about r-1 LF steps on average.     */
  int kmer_k;           /* k-mer ds-interval table (Section 2.5 precomputes all 10-mers):
                           0 = no table, 1..15 (4^k entries of 16 bytes), or -1 = automatic:
                           floor(log4 n) - 1 capped at 15, so that a k-mer occurs about 4 times
                           or more in T (15 for a 3.1 Gbp reference, 12 for 100 Mbp); the
                           value used is reported by mbw_index_info.                              */
  int bisulfite;        /* 0: T = R . revcomp(R) . $.  1: four-copy 3-base text over
                           C->T(R) . G->A(R) and its reverse complement (Section 2.9).           */
  int ref_is_codes;     /* 1: ref holds codes 0..3 (A,C,G,T); 0: ASCII (case-insensitive)      */
  uint64_t rng_seed;    /* ambiguous (non-ACGT) reference bases become random bases drawn from
                           SplitMix64 seeded with this value (Section 2.1)                       */
  int device;           /* HIP device ordinal that will hold the index                          */
  int isa_sample;       /* 0: none.  q >= 1: also keep the packed text T (2 bits per symbol) and the
                           inverse suffix array at text positions that are multiples of q (1..64),
                           which let the seeding kernels extend a match that occurs once by
                           comparing it with the text (same results, fewer index accesses).      */
  int sb_lines_log2;    /* occurrence lines per superblock as a power of two: 0 = the default 2^23
                           (each superblock spans 3.2 G rows of B, so a 3.1 Gbp plain index has 2 and
                           a bisulfite one 4); 1..23 smaller, for tests that need several
                           superblocks on a small reference.  An index may have at most 8.        */
} mbw_build_opts;

/* Build the index of `ref` (host pointer, `len` bases, 1 <= len < 2^38) on the GPU and keep it
 * resident in that device's HBM.  Builds T, sorts its suffixes on the GPU, derives B, the
 * occurrence lines (Section 2.2), the sampled SA (Section 2.4) and the optional k-mer table.
 * The caller keeps ownership of `ref`; *out is owned by the caller and released with
 * mbw_index_free.  Blocking.  Errors: MBW_E_INVAL (len, options), MBW_E_NOMEM, MBW_E_HIP.      */
int mbw_index_build(const uint8_t *ref, uint64_t len, const mbw_build_opts *opts, mbw_index **out);

/* mbw_index_build from a FASTA file: R is the sequences of its records back to back (headers start
 * with '>', a record's name is its header up to the first blank; line breaks and blanks inside
 * sequences are dropped; every other character is a base, ambiguous ones drawn as for
 * mbw_index_build).  The records are kept with the index (mbw_index_contig) and in its file.
 * opts->ref_is_codes must be 0.  Errors: MBW_E_IO (open, read), MBW_E_FORMAT (no record, sequence
 * before the first header, a record without sequence), and those of mbw_index_build. */
int mbw_index_build_fasta(const char *fasta_path, const mbw_build_opts *opts, mbw_index **out);

/* The records of the index's reference: an index built from memory has one, with an empty name,
 * covering R; a FASTA build has the file's.  mbw_index_contig gives record i (name valid while the
 * index lives; start and length in R coordinates); mbw_ref_to_contig maps a position of R (e.g.
 * from mbw_pos_to_ref) to its record and the offset in it.  Errors: MBW_E_INVAL. */
int mbw_index_contigs(const mbw_index *idx, uint64_t *n);
int mbw_index_contig(const mbw_index *idx, uint64_t i, const char **name, uint64_t *start, uint64_t *len);
int mbw_ref_to_contig(const mbw_index *idx, uint64_t ref_pos, uint64_t *contig, uint64_t *offset);

/* Write the resident index to `path` (versioned header + checksummed arrays + the record table),
 * streamed through 128 MiB of pinned host memory.  Blocking.  Errors: MBW_E_IO, MBW_E_NOMEM, MBW_E_HIP. */
int mbw_index_save(const mbw_index *idx, const char *path);

/* Read an index file written by mbw_index_save and make it resident on `device`, streamed
 * through 128 MiB of pinned host memory.  Before anything is allocated the header must pass the
 * builder's limits (n < 2^39, n = 2|R|+1 or 4|R|+1, primary < n, C non-decreasing with C[$] = 0,
 * C[A] = 1 and C[T] <= n, at most 8 superblocks, array sizes consistent) and the file size must
 * equal what the header states; the record table must cover R exactly.
 * Errors: MBW_E_IO, MBW_E_FORMAT (magic, version, fields, sizes or checksum), MBW_E_NOMEM, MBW_E_HIP. */
int mbw_index_load(const char *path, int device, mbw_index **out);

/* Release the index.  Contexts and servers keep the index they were created on: an index freed
 * while any of them is alive is released when the last of them is freed or closed (device memory
 * is never freed under a kernel that reads it). */
void mbw_index_free(mbw_index *idx);

typedef struct {
  uint64_t n;              /* |T| */
  uint64_t len_r;          /* |R| (original reference length) */
  uint64_t primary;        /* the row x with S(x) = 0 (B[x] = $) */
  uint64_t n_lines;        /* occurrence lines (128 bytes each) */
  uint64_t bytes_resident; /* device bytes held by the index */
  uint64_t C[5];           /* C[a] = |{i : B[i] < a}| for a = $, A, C, G, T (C[0] = 0)         */
  int bases_per_line;      /* rows of B per occurrence line (384) */
  int line_bytes;          /* 128 */
  int sa_sample;
  int kmer_k;
  int bisulfite;
  int device;
  int isa_sample;          /* 0 when the index holds no text / inverse-SA samples */
  int sb_lines_log2;       /* occurrence lines per superblock = 2^sb_lines_log2 */
  int n_superblocks;
} mbw_index_info_t;

int mbw_index_info(const mbw_index *idx, mbw_index_info_t *out);

/* Device pointers to the resident arrays (read-only views for tests and tools):
 * lines: n_lines x 128 B; each line = u32 counts of A, C, G in B from the start of its superblock
 *        (2^sb_lines_log2 lines) to the line (the $ row counted as A), five u32 sub-checkpoints (counts of A,
 *        C, G in the line's first 64, 128, 192, 256, 320 rows, 9 bits each at bits 0, 9, 18),
 *        then the line's six 64-row blocks, each a u64 of the low code bits and a u64 of the high
 *        code bits (row t of the block at bit t; the $ row holds A).
 * ssa:   ceil(n/r) x u64, ssa[x/r] = S(x).
 * kmer:  4^k x 16 B packed (k:40 | k':40 | s:40 bits, little-endian), code = sum P[q]*4^q. */
int mbw_index_device_arrays(const mbw_index *idx, const void **lines, const void **ssa, const void **kmer);
/* Device pointer to the superblock table the kernels read (read-only view): for each of the
 * n_superblocks superblocks of 2^sb_lines_log2 lines, 8 x u64: the counts of A, C, G, T in B
 * before its first row (the $ row counted as A), then for c = A, C, G, T the sum of those counts
 * over the symbols after c. */
int mbw_index_superblock_table(const mbw_index *idx, const void **sbtab);

/* ---- seeding ------------------------------------------------------------------------------ */
typedef struct mbw_ctx mbw_ctx;

/* A context owns the device work space and result buffers for one stream of mbw_seed calls.
 * Contexts are not thread-safe; use one per host thread / stream.  A context keeps its index alive
 * until it is freed.
 * mbw_ctx_free waits for all work on the context's device (so it is safe after a call that failed
 * part way, and the caller's last stream need not exist any more), frees the work space on a
 * stream of the context's own and trims the device's memory pool. */
int mbw_ctx_create(const mbw_index *idx, mbw_ctx **out);
void mbw_ctx_free(mbw_ctx *ctx);

typedef struct {
  int min_occ;        /* c of the (l,c)-SMEMs (Section 2.1); >= 1; 1 for plain seeding (Section 2.6) */
  int reseed;         /* second seeding round (Section 2.6): for each round-1 SMEM [i,j) with
                         j-i >= reseed_len and s <= reseed_occ, the (floor((j-i)/2), s+1)-SMEMs of
                         P[i,j); duplicates removed */
  int reseed_len;     /* 38 in the paper */
  int reseed_occ;     /* 10 in the paper */
  int bs_role;        /* bisulfite index only: 1 = read 1 (C->T, keep positions in the forward
                         C->T and reverse G->A copies), 2 = read 2 (G->A, keep forward G->A and
                         reverse C->T) (Section 2.9); 0 = plain */
  int kernel;         /* MBW_KERNEL_COOP (default: persistent wave kernels) or MBW_KERNEL_PLAIN
                         (one read per thread running the serial algorithm; the baseline) */
  int use_kmer;       /* use the index's k-mer table (wave kernels) */
  int blocks_per_cu;  /* persistent grid size per compute unit (wave kernels): > 0 that many (at
                         most the occupancy limit), -1 the occupancy limit, 0 sized per launch by
                         its work (about one block per CU per 1,200 round-1 queries, 4,000
                         round-2 queries or 24,000 positions to locate, up to the occupancy
                         limit, and up to 4 blocks for locate: small batches run faster on fewer
                         waves, and locate on large ones with 4 waves per SIMD rather than 8) */
  int no_stage;       /* 1: do not stage reads of <= 160 bases in LDS */
  int unique_ext;     /* 1: when the index holds the text and inverse-SA samples, a forward
                         extension whose interval has s = 1 continues by comparing the read with
                         the text at the match's single position (wave kernels; same results) */
  int seg_len;        /* queries longer than this many bases (and reads too long for the LDS
                         staging area) are split into segments seeded by separate lanes
                         (wave kernels; same results); 0 = 256, minimum 32 */
  int bs_refine;      /* bisulfite only (needs bs_role): refine every kept (seed, position) pair
                         as in Section 2.9 into mbw_result.pieces */
  int wave_chunk;     /* reads (queries) a wave of the SMEM kernels takes from the work queue at a
                         time (wave kernels; same results): 0 = automatic (as many as leave every
                         wave of the grid about 8 takes, at most 256), else 1..256 fixed (a fixed
                         size leaves waves of the grid idle on a batch of fewer than that many reads
                         per wave) */
  int unique_defer;   /* with unique_ext, for reads staged in LDS (round 1): 1 = a lane whose forward
                         extension reaches s = 1 hands the match to a task list and takes the next
                         read; a continuation kernel finishes the listed matches against the text
                         and lists their reads for another pass, and the passes alternate until
                         every read is done (same results; the SMEM kernel runs without the
                         unique-match stages, about a third fewer vector instructions, but the
                         passes serialise the continuation work that the lanes otherwise overlap
                         with extension, and each pass costs the host two waits: slower on the
                         150 bp reads measured); 0 = the lane finishes the match itself */
} mbw_seed_opts;


#define MBW_KERNEL_COOP  0
#define MBW_KERNEL_PLAIN 1

/* One seed = one (l,c)-SMEM P[qbeg, qend) of read `read_id` with its ds-interval (k, kr, s).
 * Its reference positions (T coordinates, 0 <= pos < n-1) are pos[pos_off .. pos_off+npos).
 * flags bit 0 (MBW_SEED_UNLOCATED): s > max_occ, positions not computed (npos = 0).
 * flags bit 1 (MBW_SEED_ROUND2): found in the second seeding round. */
typedef struct {
  uint32_t read_id, qbeg, qend, flags;
  uint64_t k, kr, s;
  uint64_t pos_off;
  uint32_t npos, reserved;
} mbw_seed_t;

#define MBW_SEED_UNLOCATED 1u
#define MBW_SEED_ROUND2    2u

/* A refined bisulfite seed match (Section 2.9): the kept (seed, position) pair of seed `seed` split
 * at the bases where the original read has a C over an original reference T (read 1; read 2: G
 * over A), which bisulfite conversion cannot explain; each piece of at least min_seed_len bases
 * is P[qbeg, qend) of read read_id at text position pos.  The original reference base under text
 * position t is R[t mod |R|] for t < 2|R| and the complement of R[(4|R| - 1 - t) mod |R|] above. */
typedef struct {
  uint32_t read_id, qbeg, qend, seed;
  uint64_t pos;
} mbw_piece_t;

typedef struct {
  uint64_t n_seeds;
  uint64_t n_pos;
  const mbw_seed_t *seeds; /* device pointer, n_seeds records sorted by (read_id, qbeg, qend)     */
  const uint64_t *pos;     /* device pointer, n_pos positions; within a seed in SA-row order      */
  uint64_t lines_smem;     /* algorithmic 128-B index lines touched by SMEM finding (counted)    */
  uint64_t lines_locate;   /* ... by locate (LF steps + SA-sample reads)                          */
  uint64_t steps;          /* extension steps (Algorithm 1 calls) */
  uint64_t lf_steps;       /* LF steps in locate */
  float ms_smem;            /* device time of the SMEM kernel launches (HIP events around each) */
  float ms_locate;          /* device time of the locate kernel launch */
  float ms_total;           /* device time of the whole call */
  int n_smem_launches;      /* SMEM kernel launches in this call (per round and length bin) */
  uint64_t wave_iters;      /* diagnostics of the wave kernels: loop iterations summed over waves, */
  uint64_t lane_iters;      /* and lane iterations that held a query (utilisation = lane / 64 wave) */
  uint64_t max_chain;       /* the most iterations one query took (wave kernels) */
  uint64_t n_pieces;        /* bs_refine: refined pieces (device pointer, in seed and position order) */
  const mbw_piece_t *pieces;
} mbw_result;

/* Seed a batch of reads: for every read P, its (l,c)-SMEMs (Section 2.1 definitions; found with
 * Algorithm 3, BatchFindSMEM, Section 2.5, with the k-mer shortcut), the second seeding round of
 * Section 2.6 ((floor((j-i)/2), s+1)-SMEMs inside long rare SMEMs), and the reference positions of
 * every seed with s <= max_occ by LF walks to the sampled SA (Algorithm 2, Section 2.4); for a
 * bisulfite index the strand filter and optional refinement of Section 2.9.
 *   reads:   concatenated read bases, ASCII (A/C/G/T case-insensitive; anything else is a base
 *            that matches nothing), host or device pointer.
 *   lengths: n_reads x u32 read lengths (host or device), each < 65536; reads are stored back to
 *            back in `reads` in this order.
 *   min_seed_len: l >= 1.  max_occ >= 1: seeds with s > max_occ are reported but not located.
 *   stream:  hipStream_t to run on (NULL = default stream).
 * The call runs on `stream` and waits for it before returning (the result counts are needed on
 * the host).  Results stay in device memory owned by `ctx` and remain valid until the next
 * mbw_seed on the same ctx.  Errors: MBW_E_INVAL, MBW_E_NOMEM, MBW_E_HIP. */
int mbw_seed(mbw_ctx *ctx, const uint8_t *reads, const uint32_t *lengths, uint64_t n_reads,
             int min_seed_len, int max_occ, const mbw_seed_opts *opts, void *stream, mbw_result *out);

/* Caller-owned buffers of mbw_seed_into (device memory, e.g. torch tensors), and the sizes the call
 * needs, written back by it. */
typedef struct {
  void *workspace;              /* every temporary of the call is carved from here; 256-byte aligned */
  uint64_t workspace_bytes;
  mbw_seed_t *seeds;            /* result records */
  uint64_t seeds_cap;
  uint64_t *pos;                /* positions */
  uint64_t pos_cap;
  mbw_piece_t *pieces;          /* refined pieces (opts.bs_refine only; may be NULL otherwise) */
  uint64_t pieces_cap;
  uint64_t workspace_needed;    /* written back: work space bytes used, or at least needed */
  uint64_t seeds_needed, pos_needed, pieces_needed;   /* written back once known */
} mbw_seed_buffers;

/* mbw_seed with caller-owned memory: computes exactly what mbw_seed computes (Algorithm 3 for the
 * (l,c)-SMEMs of Section 2.5, the two seeding rounds of Section 2.6, Algorithm 2's locate of Section
 * 2.4, the bisulfite filter and refinement of Section 2.9) but allocates no device memory: all work
 * buffers come from bufs->workspace and the seeds, positions and pieces are written to the caller's
 * buffers, which the returned mbw_result points to (valid while the caller keeps them).  The context
 * must be the one whose index is meant; its own buffers are left untouched.
 * A buffer that is too small makes the call return MBW_E_CAPACITY with the sizes learnt so far in
 * bufs->*_needed (a work space shortfall reports at least the bytes asked for); enlarging those
 * buffers and calling again converges (each retry gets further).  On success the *_needed fields
 * hold the exact sizes used.  Errors: as mbw_seed, plus MBW_E_CAPACITY. */
int mbw_seed_into(mbw_ctx *ctx, const uint8_t *reads, const uint32_t *lengths, uint64_t n_reads, int min_seed_len,
                  int max_occ, const mbw_seed_opts *opts, void *stream, mbw_seed_buffers *bufs, mbw_result *out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): mbw_seed_into with the work space replaced by a static device
 * array of 128 MiB that the library holds on each GPU it runs on until the process ends; the call
 * allocates nothing (no hipMalloc, hipFree, pinned memory or library allocation).  reads and
 * lengths must be in device memory; the seeds, positions and pieces go to the caller's buffers
 * as for mbw_seed_into (bufs->workspace and workspace_bytes are ignored).  A batch whose work space
 * does not fit in the 128 MiB (a few tens of thousands of 150-base reads) is refused with
 * MBW_E_CAPACITY, a message saying so and the size it needs in bufs->workspace_needed.  Every call
 * on one GPU shares that GPU's array: calls that overlap on a GPU (other threads, other streams)
 * race and must be serialised by the caller.  Errors: as mbw_seed_into. */
int mbw_seed_static(mbw_ctx *ctx, const uint8_t *reads, const uint32_t *lengths, uint64_t n_reads, int min_seed_len,
                    int max_occ, const mbw_seed_opts *opts, void *stream, mbw_seed_buffers *bufs, mbw_result *out);

/* ---- captured graphs -------------------------------------------------------------------- */
/* The seeding path of mbw_seed (Algorithm 3 of Section 2.5 in both rounds of Section 2.6, then
 * Algorithm 2 of Section 2.4), recorded once as a HIP graph over device buffers sized by a plan and
 * replayed for every batch, with the same length bins as mbw_seed (reads of at most 160 bases
 * staged in LDS; longer ones, when the plan allows them, in segments): each call copies the batch in,
 * launches the graph and waits once (mbw_seed waits for every intermediate count).  Same seeds and
 * positions as mbw_seed with the same options.  Sorts and scans span the plan's capacities, so a
 * plan much larger than its batches costs time.  A graph belongs to one context, is freed before
 * it and is used by one host thread at a time; it keeps its index alive. */
typedef struct mbw_graph mbw_graph;
typedef struct {
  uint64_t max_reads;       /* reads per batch at most (>= 1, < 2^31) */
  uint64_t max_bases;       /* bases per batch at most; 0 = max_read_len per read */
  uint64_t max_seeds;       /* seed records before duplicates are dropped; 0 = 8 per read (output
                               slack of the kernels' per-wave chunks is added) */
  uint64_t max_subqueries;  /* re-seeding queries; 0 = 2 per read (plus the same slack) */
  uint64_t max_positions;   /* positions; 0 = 64 per read */
  uint64_t max_read_len;    /* longest read; 0 = 160 (the staged bin only); at most 65535.  Longer
                               reads add the unstaged bin: segments of seg_len bases, at most
                               max_bases / seg + max_reads in round 1 and max_subqueries +
                               4 max_bases / seg in round 2 */
  uint64_t max_pieces;      /* bs_refine: refined pieces; 0 = max_positions */
} mbw_graph_plan;
/* Allocate the plan's buffers on the context's device (mbw_graph_info reports the capacities with
 * slack) and capture the graph.  opts as for mbw_seed, bisulfite roles and refinement included
 * (the strand filter and the refinement run inside the graph); the plain kernel, no_stage and
 * unique_defer are refused (MBW_E_INVAL).  Errors:
 * MBW_E_INVAL, MBW_E_NOMEM, MBW_E_HIP (capture or instantiation failed). */
int mbw_graph_create(mbw_ctx *ctx, const mbw_graph_plan *plan, int min_seed_len, int max_occ,
                     const mbw_seed_opts *opts, mbw_graph **out);
int mbw_graph_info(const mbw_graph *g, mbw_graph_plan *plan);   /* capacities, slack included */
/* Seed one batch (reads and lengths on the host or the device, as for mbw_seed) on `stream`;
 * blocking.  The result points into the graph's buffers and stays valid until the graph's next
 * call or mbw_graph_free; mbw_result_download with the graph's context copies it out.  ms_total is
 * the graph's device time (ms_smem and ms_locate are not split out).  Errors: MBW_E_INVAL (more
 * reads or bases than the plan, a read longer than its max_read_len), MBW_E_CAPACITY (the batch
 * needs more seed, sub-query, segment, position or piece slots than the plan holds: the message gives the
 * counts; seed it with mbw_seed or a larger plan), MBW_E_HIP. */
int mbw_graph_seed(mbw_graph *g, const uint8_t *reads, const uint32_t *lengths, uint64_t n_reads, void *stream,
                   mbw_result *out);
void mbw_graph_free(mbw_graph *g);

/* Copy a result to host buffers (seeds: n_seeds records, pos: n_pos values; either may be NULL). */
int mbw_result_download(mbw_ctx *ctx, const mbw_result *res, mbw_seed_t *seeds, uint64_t *pos);
/* Copy the refined bisulfite pieces of a result (bs_refine) to host memory (n_pieces records). */
int mbw_result_download_pieces(mbw_ctx *ctx, const mbw_result *res, mbw_piece_t *pieces);

/* Autotuner for the wave kernels: runs mbw_seed on this batch with candidate schedules (length
 * binning on or off, segment lengths 128/256/1024, persistent blocks per CU, i.e. the waves each
 * CU keeps in flight, sized by the work, at the occupancy limit or 2, unique-match extension on or
 * off), each once untimed and once timed, then with the best of those the reads a wave takes from
 * the work queue at a time (16, 64, 256 against automatic), and writes the fastest to *best (other
 * fields copied from *base, or the defaults when base is NULL) and its device time to *best_ms.  Every candidate yields the same seeds.  Blocking; uses ctx's buffers
 * (its last result is overwritten).  Errors: as mbw_seed. */
int mbw_tune(mbw_ctx *ctx, const uint8_t *reads, const uint32_t *lengths, uint64_t n_reads, int min_seed_len,
             int max_occ, const mbw_seed_opts *base, void *stream, mbw_seed_opts *best, float *best_ms);

/* Map a T position of a match of length len to (strand, reference position): pos < |R| is the
 * forward strand at pos; otherwise the reverse strand at 2|R| - pos - len.  (Bisulfite index:
 * the four copies of length |R| map to their source coordinates likewise.) */
int mbw_pos_to_ref(const mbw_index *idx, uint64_t pos, uint32_t len, int *strand, uint64_t *ref_pos);

/* ---- mate-rescue prefilter (Section 2.7) -----------------------------------------------------
 * For a read P and a reference window W, M_t is the number of pairs (i, j) with
 * P[i, i+q) = W[j, j+q) and j - i = t; max_t M_t approximates the best ungapped alignment of P in
 * W, and a candidate goes on to Smith-Waterman only when max_t M_t >= min_hits.  A q-mer of P that
 * holds a base other than A/C/G/T matches nothing. */

/* One candidate: read `read_id` of the batch against the window T[win_beg, win_beg + win_len) of
 * the index text (T coordinates as for positions; the window may not reach the sentinel:
 * win_beg + win_len <= n - 1). */
typedef struct {
  uint32_t read_id;
  uint32_t win_len;
  uint64_t win_beg;
} mbw_rescue_cand_t;

/* Per candidate: max_hits = max_t M_t; best_t = the smallest t (-(|P|-q) <= t <= |W|-q) with
 * M_t = max_hits, or 0 when max_hits = 0 (also when |P| < q or |W| < q). */
typedef struct {
  uint32_t max_hits;
  int32_t best_t;
} mbw_rescue_hit_t;

typedef struct {
  int q;          /* q-mer length, 1..15 (7 in the paper) */
  int min_hits;   /* pass threshold on max_t M_t (10 in the paper), >= 0 */
  int bs_role;    /* bisulfite index only: 1 converts C->T in the read, 2 G->A (as for seeding) */
} mbw_rescue_opts;

typedef struct {
  uint64_t n_cands;
  uint64_t n_pass;
  const mbw_rescue_hit_t *hits;   /* device pointer, n_cands records in candidate order */
  const uint32_t *pass;           /* device pointer, n_pass candidate indices (ascending) with
                                     max_hits >= min_hits */
  float ms_kernel;                /* device time of the prefilter kernel (HIP events) */
  float ms_total;                 /* device time of the whole call */
} mbw_rescue_result;

/* Run the prefilter over a batch of candidates.
 *   reads, lengths, n_reads: as for mbw_seed (ASCII, host or device).  Reads are limited by the
 *            device's LDS: 3|P|/2 rounded up to a power of two, plus |P| + |W|, 32-bit words
 *            per wave must fit in 64 KiB (about |P| <= 2000 with |W| <= 8000).
 *   cands:   n_cands candidates (host or device), n_cands < 2^31.
 *   opts:    NULL = q 7, min_hits 10, no conversion.
 * The index must hold the packed text (built with isa_sample > 0, the default).  Results stay in
 * device memory owned by ctx until the next mbw_rescue_filter on it; a seeding result of the same
 * ctx is left intact.  Blocking on `stream` (the pass count is needed on the host).
 * Errors: MBW_E_INVAL (q, min_hits, bs_role, a read_id >= n_reads, a window outside the text, an
 * index without text, sizes beyond the LDS limit), MBW_E_NOMEM, MBW_E_HIP. */
int mbw_rescue_filter(mbw_ctx *ctx, const uint8_t *reads, const uint32_t *lengths, uint64_t n_reads,
                      const mbw_rescue_cand_t *cands, uint64_t n_cands, const mbw_rescue_opts *opts, void *stream,
                      mbw_rescue_result *out);

/* Copy a prefilter result to host buffers (hits: n_cands records, pass: n_pass indices; either
 * may be NULL). */
int mbw_rescue_download(mbw_ctx *ctx, const mbw_rescue_result *res, mbw_rescue_hit_t *hits, uint32_t *pass);

/* ---- chaining (Section 2.6) -------------------------------------------------------------------
 * minibwa chains its variable-length seeds with minimap2's chaining (Li 2018), adapted to seeds of
 * different lengths, and keeps up to 50 chains per read.  Every located (seed, position) pair of a
 * seeding result is an anchor: span w = qend - qbeg, end (x, y) = (pos + w - 1, qend - 1), copy
 * g = x / |R| (0 forward, 1 reverse strand; 0..3 for a bisulfite index).  A read's anchors are
 * ordered by (x, y, w), and (all integers)
 *   f(i) = max(w_i, max_j f(j) + alpha(j,i) - beta(j,i))
 * over the max_pred anchors j before i with g_j = g_i, x_j < x_i, y_j < y_i, x_i - x_j <= max_gap
 * and y_i - y_j <= max_gap; alpha = min(x_i - x_j, y_i - y_j, w_i), beta = gamma(|dy - dx|),
 * gamma(0) = 0, gamma(l) = floor(l * wbar / 100) + floor(floor(log2 l) / 2), wbar = the read's
 * mean anchor span rounded down.  The predecessor of i is the nearest j reaching the maximum when
 * it exceeds w_i.  Anchors are then taken in order of descending f (equal f: earlier first); from
 * each unused one the predecessors are followed, marking anchors used, until there is none or the
 * next is used; the chain scores f(end) minus f of the used anchor where it stopped.  Chains scoring
 * at least min_score are ranked by score (equal: earlier end first) and the first max_chains kept. */
typedef struct {
  int max_gap;      /* G, >= 1 (5000) */
  int max_pred;     /* h: predecessors looked at, 1..64 (50) */
  int max_chains;   /* chains kept per read, 1..64 (50, Section 2.6) */
  int min_score;    /* (19) */
} mbw_chain_opts;

typedef struct {
  uint32_t read_id, n_anchors;
  int32_t score;
  uint32_t copy;          /* g of its anchors */
  uint64_t anchor_off;    /* its anchors: anchors[anchor_off .. anchor_off + n_anchors), ascending */
} mbw_chain_t;

typedef struct {
  uint32_t qbeg, qend;    /* the seed P[qbeg, qend) */
  uint64_t pos;           /* its text position (T coordinates) */
} mbw_anchor_t;

typedef struct {
  uint64_t n_chains;
  uint64_t n_anchors;              /* anchors in the kept chains */
  uint64_t n_input_anchors;        /* located (seed, position) pairs chained */
  const mbw_chain_t *chains;       /* device pointer: by read, then rank */
  const mbw_anchor_t *anchors;     /* device pointer */
  float ms_kernel;                 /* device time of the chaining kernel (the recurrence and extraction) */
  float ms_total;                  /* device time of the whole call (anchors, sorts, chaining, output) */
  uint64_t max_read_anchors;       /* the most anchors one read has */
  uint64_t reads_over_lds;         /* reads with more than 1,024 anchors (chained from global memory) */
} mbw_chain_result;

/* Chain the seeds of a seeding result whose arrays are in device memory (an mbw_seed result:
 * seeds sorted by read, each seed's positions at pos[pos_off ..]; every read_id < n_reads).  opts
 * NULL = the defaults above.  The result stays in device memory owned by ctx until the next
 * mbw_chain on it (a seeding or prefilter result of ctx is left intact).  Blocking on `stream`.
 * Errors: MBW_E_INVAL (options, sizes, a seed with read_id >= n_reads), MBW_E_NOMEM, MBW_E_HIP. */
int mbw_chain(mbw_ctx *ctx, const mbw_result *seeds, uint64_t n_reads, const mbw_chain_opts *opts, void *stream,
              mbw_chain_result *out);
/* Copy a chaining result to host buffers (n_chains and n_anchors records; either may be NULL). */
int mbw_chain_download(mbw_ctx *ctx, const mbw_chain_result *res, mbw_chain_t *chains, mbw_anchor_t *anchors);

/* ---- debug -----------------------------------------------------------------------------------
 * Cap the device work space every context may hold (bytes; 0 = no cap, the default).  A call that
 * would grow a context beyond it fails with MBW_E_NOMEM and leaves the context usable; a serve
 * arena larger than the cap makes mbw_serve_open fail with MBW_E_NOMEM.  For tests of allocation
 * failure.  Process-wide. */
int mbw_debug_set_mem_limit(uint64_t bytes);

/* ---- serving -------------------------------------------------------------------------------
 * A request loop over one resident index (the streaming use of Section 2.9's bisulfite mode, and
 * of plain seeding).  n_workers threads each own a seeding context, a HIP stream and a fixed device
 * arena (work space plus result buffers) allocated at mbw_serve_open: a running server allocates no
 * device memory.  Admission is by device memory: a request whose estimated work space (the seeding
 * path's sizing model for its reads and bases) exceeds one worker's arena, or that is over the
 * batch budget by itself, is refused with MBW_E_CAPACITY; a free worker takes queued requests in
 * arrival order into one device batch while the batch's estimate fits its arena (and within
 * max_batch_reads / max_batch_bases / 65536 requests), so requests that arrive while other batches
 * run join the next batch at once, and the batches of different workers overlap on the device.  A
 * batch that still runs short of its arena, or meets an allocation failure, is split in two and
 * each half run again, down to single requests, so a request's outcome never depends on what it
 * was batched with: each request's result equals what mbw_seed returns for that request alone
 * (read ids relative to the request). */
typedef struct mbw_server mbw_server;

typedef struct {
  int n_workers;              /* batches in flight at once (1..8); each worker has its own stream,
                                 and a process gets a few hardware queues (4 on MI355X by default),
                                 so more workers than that share them */
  uint64_t max_batch_reads;   /* batch budget: reads (< 2^31) ... */
  uint64_t max_batch_bases;   /* ... and bases */
  uint64_t max_queued_bases;  /* host back-pressure: submit returns MBW_E_BUSY when the queue is not
                                 empty and would exceed this many bases */
  int min_seed_len, max_occ;  /* as mbw_seed */
  mbw_seed_opts opts;         /* as mbw_seed */
  int device;                 /* must be the index's device */
  uint64_t device_bytes;      /* device memory of all worker arenas together, split evenly; 0 = each
                                 arena sized by the model for a full batch of max_batch_reads reads
                                 and max_batch_bases bases.  An arena must admit one read of 65535
                                 bases (about 100 MB; the error message gives the least size) */
} mbw_serve_cfg;

typedef struct {
  uint64_t n_seeds, n_pos;
  const mbw_seed_t *seeds;    /* host memory owned by the server until mbw_serve_release; read_id
                                 counts from the request's first read, pos_off from its first
                                 position */
  const uint64_t *pos;
  double t_submit, t_start, t_done;   /* seconds since mbw_serve_open (steady clock) */
  uint64_t batch_id, batch_reads;     /* the device batch that carried the request (the last one
                                         tried when it was split) */
  uint64_t n_pieces;          /* opts.bs_refine: the request's refined pieces (host memory owned by
                                 the server), read_id and seed counted from the request's own */
  const mbw_piece_t *pieces;
  uint32_t attempts;          /* device batches the request was part of (> 1 after a split) */
  uint32_t reserved;
} mbw_serve_result;

typedef struct {
  uint64_t batches;           /* device batches run (split halves included) */
  uint64_t batch_reads;       /* reads in them */
  uint64_t queued;            /* requests waiting for a worker */
  uint64_t split_retries;     /* batches split in two after running short */
  uint64_t failed_requests;   /* requests finished with an error */
  uint64_t device_bytes;      /* device memory held by the worker arenas */
  uint64_t workspace_bytes;   /* one worker's work space, the admission bound */
  uint64_t seeds_cap, pos_cap, pieces_cap;   /* one worker's result buffers (records) */
} mbw_serve_stats_t;

/* Start the workers and allocate their arenas.  The server keeps the index alive until it closes.  Errors:
 * MBW_E_INVAL (configuration, device_bytes below the minimum), MBW_E_NOMEM (arena or pinned
 * staging allocation, or an arena over the debug cap), MBW_E_HIP. */
int mbw_serve_open(const mbw_index *idx, const mbw_serve_cfg *cfg, mbw_server **out);
/* Queue a request (host pointers, copied before return; lengths < 65536).  Non-blocking.
 * Errors: MBW_E_INVAL, MBW_E_CAPACITY (the request can never fit a worker: see above), MBW_E_BUSY
 * (queue full: retry later), MBW_E_NOMEM. */
int mbw_serve_submit(mbw_server *s, const uint8_t *reads, const uint32_t *lengths, uint64_t n_reads,
                     uint64_t *ticket);
/* mbw_serve_submit without the host copy: the caller keeps reads and lengths valid and unchanged
 * until mbw_serve_wait reports the request finished (or the server is closed). */
int mbw_serve_submit_nocopy(mbw_server *s, const uint8_t *reads, const uint32_t *lengths, uint64_t n_reads,
                            uint64_t *ticket);
/* Wait up to timeout_ms (< 0: forever) for a request; MBW_E_BUSY if it is not finished by then,
 * else its result (valid until mbw_serve_release) or its error (the timing fields and attempts
 * are filled in either case). */
int mbw_serve_wait(mbw_server *s, uint64_t ticket, int timeout_ms, mbw_serve_result *out);
/* Free a finished request's result.  Errors: MBW_E_INVAL (unknown ticket), MBW_E_BUSY (unfinished). */
int mbw_serve_release(mbw_server *s, uint64_t ticket);
/* Counters since mbw_serve_open. */
int mbw_serve_stats(mbw_server *s, mbw_serve_stats_t *out);
/* Finish every queued request, stop the workers and free the server and its arenas. */
void mbw_serve_close(mbw_server *s);

#ifdef __cplusplus
}
#endif
#endif /* MBW_H */
