/*
 * adha.h -- C-ABI of libadha: layout remaps, layout-generic section kernels
 * and two-level layout selection for record arrays on MI355X (gfx950).
 *
 * Problem statement followed (ADHA, Majeti, Meel, Barik, Sarkar, PACT 2014):
 *   section 2: a program is a sequence of "sections" (data-parallel loops);
 *   the affinity graph's nodes are the fields the sections access; a
 *   per-section layout is obtained by greedy clustering of that graph; a
 *   program layout is a shortest path over the sections with "combine"
 *   (keep one layout) and "remap" (change layout) edges, weighted from a
 *   profile of section times.
 *   section 1 and Tables 2-3: layouts are AoS, SoA and structures of
 *   clustered fields; here each group of fields is either interleaved
 *   (tile 1) or stored in tiles of T records (AoSoA).
 *
 * Conventions for every call:
 *   - Every call returns adha_status.  Out-parameters are written only on
 *     success.  Nothing is thrown across this boundary and nothing aborts.
 *     adha_last_error() returns a message for the last failing call made
 *     on the calling thread.
 *   - All arguments are validated on the host before any device work.
 *   - Device buffers are owned by the caller, passed as plain device
 *     pointers with their capacity in bytes; they must be 256-byte aligned.
 *     The library never frees them.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default
 *     stream).  Device work is enqueued on it and is asynchronous; faults
 *     and gather-index errors surface from adha_ctx_check().
 *   - Handles from *_create are released by the matching *_destroy.
 *     Layouts, sections and programs copy what they need from the struct,
 *     so a struct may be destroyed once they exist.
 *   - A context is not thread-safe; separate contexts are.
 *
 * Layout definition (byte address of field f of record r):
 *   groups are ordered by their smallest field id; fields inside a group are
 *   packed in ascending id (p_f = byte offset inside the group's record,
 *   S_g = group record bytes, e_f = element bytes);
 *   addr(r, f) = base_g + (r / T)*T*S_g + p_f*T + (r % T)*e_f;
 *   base_0 = 0, base_{g+1} = roundup(base_g + roundup(N, T_g)*S_g, 256);
 *   size = roundup(end of last group, 256); a one-field group has T = 1;
 *   bytes owned by no (r, f) are padding and a remap writes them as zero.
 */
#ifndef ADHA_H
#define ADHA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t adha_status;
#define ADHA_OK 0
#define ADHA_WARN_FALLBACK 1     /* success, but a fallback was taken */
#define ADHA_ERR_INVALID (-1)    /* bad argument; nothing was launched */
#define ADHA_ERR_OOM (-2)        /* device or host allocation failed */
#define ADHA_ERR_DEVICE (-3)     /* HIP error (launch, fault, no device) */
#define ADHA_ERR_STATE (-4)      /* object not in a usable state */
#define ADHA_ERR_UNSUPPORTED (-5)/* valid request this library cannot do */
#define ADHA_ERR_IO (-6)         /* file missing, unreadable or corrupt */

/* Element types.  Integer types are two's complement (I32, I16) or unsigned
 * (U32, U16, U8).  As a term an integer field converts to floating point
 * exactly (U8, U16, I16 always; I32 and U32 in double) or to nearest even
 * (I32 and U32 in float); in the integer fold it is its value modulo 2^32
 * (I16 sign-extended, unsigned types zero-extended).  An integer write field
 * keeps the low bytes of the fold (its value modulo 2^(8 e)). */
typedef enum {
  ADHA_F32 = 0, ADHA_F64 = 1, ADHA_I32 = 2, ADHA_RAW = 3,
  ADHA_U32 = 4, ADHA_U8 = 5, ADHA_U16 = 6, ADHA_I16 = 7
} adha_dtype;

/* Section bodies (the paper gives none; these are the workloads' bodies).
 * Terms are read first: direct sections (degree 0) read the read fields of
 * record i in ascending id; gather sections read, for j = 0..d-1, the read
 * fields in ascending id of record idx[i*d + j].  Then each write field w_k
 * (ascending id, k < 2) of record i is written:
 *   GEN, fp w:  acc = 0, per term v = convert(t) to w's type (int -> fp and
 *               f64 -> f32 round to nearest even), k = 0: acc = acc + v,
 *               k = 1: acc = acc*0.5 + v, every operation rounded in w's type;
 *   GEN, integer w: acc = 0, per term u = its 32-bit pattern (f64: low ^
 *               high; an integer term its value mod 2^32), k = 0: acc = acc + u,
 *               k = 1: acc = (acc ^ u) * 16777619 (mod 2^32), stored as the low
 *               bytes that fit w;
 *   MULADD3:    w = a*b + c (two roundings), read set {a < b < c}, direct only;
 *   SUB2:       w = a - b, read set {a < b}, direct only;
 *   SUM:        w = ((t0 + t1) + ...) left to right, direct only.
 * MULADD3, SUB2 and SUM need one fp write field.  Fields of 1 and 2 bytes, and
 * fields that a layout places at addresses that are not multiples of 4, are
 * read and written byte by byte (a slower kernel form). */
typedef enum {
  ADHA_OP_GEN = 0,
  ADHA_OP_MULADD3 = 1,
  ADHA_OP_SUB2 = 2,
  ADHA_OP_SUM = 3,
  ADHA_OP_REDUCE = 4 /* a reduction over the records: adha_section_create_reduce */
} adha_op;

#define ADHA_MAX_FIELDS 64
#define ADHA_MAX_READ 32
#define ADHA_MAX_WRITE 2
#define ADHA_MAX_DEGREE 32
#define ADHA_MAX_TILE 256
#define ADHA_MAX_SECTIONS 64
#define ADHA_MAX_REDUCE_CELLS 4096 /* n_keys * (n_read + 1) of a reduction */

typedef struct adha_ctx adha_ctx;
typedef struct adha_struct adha_struct;
typedef struct adha_layout adha_layout;
typedef struct adha_section adha_section;
typedef struct adha_program adha_program;
typedef struct adha_plan adha_plan;

/* ------------------------------------------------------------ errors */
/* Static text for a status code. */
const char *adha_status_string(adha_status st);
/* Message of the last failing call on this thread ("" if none). */
const char *adha_last_error(void);
/* Library version, major*10000 + minor*100 + patch. */
int32_t adha_version(void);

/* ------------------------------------------------------------ context */
/* Opens `device` (must be a gfx950 GPU).  Owns caches of kernel descriptors
 * and the cost model.  ERR_DEVICE if the device is missing or not gfx950. */
adha_status adha_ctx_create(int32_t device, adha_ctx **out);
adha_status adha_ctx_destroy(adha_ctx *ctx);
/* Waits for `stream`, then reports: ERR_DEVICE on a HIP error, ERR_INVALID
 * if a gather section met an index outside [0, N) or a reduction a key
 * outside [0, n_keys) since the last check (such terms or records are
 * left out), else OK.  Clears that flag. */
adha_status adha_ctx_check(adha_ctx *ctx, void *stream);
/* Number of compute units (used to size persistent launches). */
adha_status adha_ctx_cu_count(const adha_ctx *ctx, int32_t *out);

typedef enum {
  /* 1 (default): a gather whose read fields share one interleaved group
   * fetches each neighbour's span with wide loads, and direct sections over
   * mixed F32 / F64 / I32 / U32 fields, direct sections with a narrow or
   * unaligned field and stencils with a narrow or unaligned read field (up
   * to 8 reads) take the kernels specialised on the write types; 0: one
   * load per field and the generic kernels (same results). */
  ADHA_OPT_SPAN_GATHER = 1,
  /* reductions: workgroups per compute unit in the first pass (1..32,
   * default 8) */
  ADHA_OPT_REDUCE_WG_PER_CU = 2,
  /* reductions: 1 (default) compensated double-double sums of floating-
   * point columns; 0 plain double sums (same fixed order, faster, error up
   * to about (m-1) * 2^-53 * sum|x| for m values) */
  ADHA_OPT_REDUCE_COMPENSATED = 3,
  /* host backend threads (0: one per core, at most 64; up to 256) */
  ADHA_OPT_HOST_THREADS = 4
} adha_option;
adha_status adha_ctx_set_option(adha_ctx *ctx, adha_option opt, int64_t value);

/* ------------------------------------------------------------ struct */
/* A struct of n_records records (n_records >= 0; 0 makes every operation a
 * no-op).  Fields are added in order and get ids 0, 1, ... */
adha_status adha_struct_create(int64_t n_records, adha_struct **out);
/* dtype F32, I32 and U32 need elem_bytes 4, F64 needs 8, U16 and I16 need
 * 2, U8 needs 1, RAW any of 1, 2, 4, 8 (RAW fields can be remapped but not
 * used by sections).  At most 64 fields and 2048 record bytes. */
adha_status adha_struct_add_field(adha_struct *s, adha_dtype dt, uint32_t elem_bytes,
                                  int32_t *out_id);
adha_status adha_struct_destroy(adha_struct *s);
adha_status adha_struct_info(const adha_struct *s, int64_t *n_records, int32_t *n_fields,
                             uint32_t *record_bytes);

/* ------------------------------------------------------------ layouts */
/* group_of_field[f] is f's group label; labels must be exactly
 * 0..n_groups-1; tile_of_group[g] is a power of two in [1, 256]. */
adha_status adha_layout_create(const adha_struct *s, uint32_t n_groups,
                               const uint32_t *group_of_field, const uint32_t *tile_of_group,
                               adha_layout **out);
/* AoS: one interleaved group.  SoA: one group per field. */
adha_status adha_layout_aos(const adha_struct *s, adha_layout **out);
adha_status adha_layout_soa(const adha_struct *s, adha_layout **out);
adha_status adha_layout_destroy(adha_layout *l);
/* Bytes a buffer in this layout occupies. */
adha_status adha_layout_nbytes(const adha_layout *l, uint64_t *out);
/* Byte address of field f of record r (0 <= r < N). */
adha_status adha_layout_addr(const adha_layout *l, int64_t r, int32_t f, uint64_t *out);
/* Canonical form: group index of every field (groups ordered by smallest
 * field id) and each group's tile.  Either array may be NULL; each needs
 * room for n_fields entries. */
adha_status adha_layout_groups(const adha_layout *l, uint32_t *n_groups,
                               uint32_t *group_of_field, uint32_t *tile_of_group);
/* *out = 1 when a and b have the same struct shape and address map (the
 * same groups, tiles and group bases). */
adha_status adha_layout_equal(const adha_layout *a, const adha_layout *b, int32_t *out);
/* A placed copy of l: the same groups with explicit byte offsets bases[g]
 * (one per group in canonical group order, multiples of 256).  Group g then
 * owns the region [bases[g], bases[g] + roundup(roundup(N, T_g) * S_g, 256));
 * regions may not overlap; the layout's size is the end of the last one.
 * Bytes outside every region do not belong to the layout: remaps into it
 * leave them alone.  Used to run a program in one buffer in which groups
 * that two consecutive layouts share stay where they are. */
adha_status adha_layout_place(const adha_layout *l, uint32_t n_groups, const uint64_t *bases,
                              adha_layout **out);
/* Group bases (n_groups entries, canonical group order). */
adha_status adha_layout_bases(const adha_layout *l, uint64_t *bases);

/* ------------------------------------------------------------ remap */
/* Remap (section 2, the remap edge; section 3, the remap between the
 * Medical program's sections): writes into dst, laid out by dst_l, every
 * field of every record of src, laid out by src_l, and zero into every
 * padding byte.  Bit-exact byte copy.  Both layouts must describe the same
 * struct shape; src and dst must not overlap; caps must cover each
 * layout's size. */
adha_status adha_remap(adha_ctx *ctx, const adha_layout *src_l, const void *src, uint64_t src_cap,
                       const adha_layout *dst_l, void *dst, uint64_t dst_cap, void *stream);

/* Remap inside one buffer that moves only what changes (section 2: the
 * remap edge is weighed by the fields two layouts have in common).  Both
 * layouts describe where the struct's groups sit in buf (placed layouts,
 * or canonical ones).  A group of dst_l that src_l holds with the same
 * fields, tile and base stays untouched; every other group of dst_l is
 * written -- its fields copied from where src_l holds them, its padding
 * zeroed -- and so N * (their bytes) are read and written, where a whole
 * remap moves N * S.  All other bytes of buf keep their values.  A moving
 * group of dst_l may not overlap a group of src_l that moves
 * (ERR_INVALID, checked before any launch); buf_cap must cover both. */
adha_status adha_remap_in_place(adha_ctx *ctx, const adha_layout *src_l, const adha_layout *dst_l, void *buf,
                                uint64_t buf_cap, void *stream);

typedef struct {
  const adha_layout *src_layout;
  const void *src;
  uint64_t src_cap;
  const adha_layout *dst_layout;
  void *dst;
  uint64_t dst_cap;
} adha_remap_item;

/* flags for adha_remap_batched */
#define ADHA_BATCH_GRAPH 1u     /* capture the launches once in a hipGraph, replay after */
#define ADHA_BATCH_SEPARATE 2u  /* one adha_remap per item instead (for comparison) */

/* Remaps many arrays (each item as adha_remap) with one persistent launch
 * over a work list of record tiles, plus one launch for all ragged tails.
 * With ADHA_BATCH_GRAPH the context caches an instantiated graph keyed by
 * the item list and replays it when the same list comes again.  Items must
 * not overlap each other. */
adha_status adha_remap_batched(adha_ctx *ctx, uint32_t n, const adha_remap_item *items,
                               uint32_t flags, void *stream);

/* Tile shape used for a remap (records per tile, 16-byte slots per thread,
 * LDS padding shift); 0 in any field = choose automatically. */
typedef struct {
  uint32_t tile_records;
  uint32_t slots;
  uint32_t pad_shift;
  uint32_t wg_per_cu;
  uint32_t order;       /* 1: contiguous tile ranges per workgroup, 2: strided */
  uint32_t nontemporal; /* 1: ordinary accesses, 2: streaming (non-temporal) */
} adha_tile_shape;
/* Force a tile shape for subsequent remaps of this layout pair (tests and
 * the autotuner).  Invalid shapes are rejected with ERR_INVALID. */
adha_status adha_remap_set_shape(adha_ctx *ctx, const adha_layout *src_l, const adha_layout *dst_l,
                                 const adha_tile_shape *shape);
/* Tile shape the next remap of this pair would use. */
adha_status adha_remap_get_shape(adha_ctx *ctx, const adha_layout *src_l, const adha_layout *dst_l,
                                 adha_tile_shape *out);

/* Host-only description of how a remap would run with its default tile
 * shape on a device with cu_count compute units: no device is touched. */
typedef struct {
  adha_tile_shape shape;
  uint64_t full_tiles;        /* record tiles moved by the main kernel */
  uint64_t tail_bytes;        /* destination bytes written by the tail kernel */
  uint64_t descriptor_bytes;  /* size of the launch's descriptor blob */
  uint64_t grid;              /* workgroups of the main kernel */
  uint32_t lds_bytes;         /* LDS per workgroup of the main kernel */
  uint32_t byte_path;         /* 1: main kernel assembles dwords from bytes (1- or 2-byte fields) */
} adha_remap_info;
adha_status adha_remap_describe(const adha_layout *src_l, const adha_layout *dst_l, int32_t cu_count,
                                adha_remap_info *out);

/* Autotuner.  Times candidate tile shapes (records per tile, workgroups per
 * CU, tile order, streaming accesses) on the caller's buffers, keeps the
 * fastest for this pair and for every pair of the same class (layout kinds,
 * record bytes, largest tile, element sizes, log2 N) in the context's tuning
 * database, and reports it with its time and the default shape's time
 * (microseconds, median of reps).  dst is overwritten. */
adha_status adha_tune_remap(adha_ctx *ctx, const adha_layout *src_l, const void *src, uint64_t src_cap,
                            const adha_layout *dst_l, void *dst, uint64_t dst_cap, uint32_t reps,
                            void *stream, adha_tile_shape *best, double *best_us, double *default_us);
/* Tunes the batch policy used by adha_remap_batched (bytes per tile,
 * workgroups per CU, order, streaming) on the given items. */
adha_status adha_tune_batched(adha_ctx *ctx, uint32_t n, const adha_remap_item *items, uint32_t reps,
                              void *stream, uint32_t *tile_bytes, adha_tile_shape *best, double *best_us,
                              double *default_us);
/* Tuning database as text (one entry per line, versioned header and
 * checksum).  Loading a missing or corrupt file returns ERR_IO and leaves
 * the context's database unchanged. */
adha_status adha_tune_save(const adha_ctx *ctx, const char *path);
adha_status adha_tune_load(adha_ctx *ctx, const char *path);

/* ------------------------------------------------------------ sections */
/* A section (section 2: one data-parallel loop) reading n_read fields and
 * writing n_write fields, direct (degree 0) or gathering `degree` neighbours
 * per record through an int32 index array [N][degree].  Gather sections
 * must not write a field they read.  Ids are sorted internally.  op is
 * GEN, MULADD3, SUB2 or SUM; reductions come from adha_section_create_reduce. */
adha_status adha_section_create(const adha_struct *s, adha_op op, uint32_t n_read,
                                const int32_t *read, uint32_t n_write, const int32_t *write,
                                uint32_t degree, adha_section **out);
/* A stencil section (section 3: the Medical sections are loops over a
 * 256^3 image): a GEN gather whose d neighbours are fixed offsets on a 3-D
 * grid of nx * ny * nz records (N must equal that product; record r sits at
 * x = r % nx, y = (r / nx) % ny, z = r / (nx * ny)).  Neighbour j of r is
 * the record at (x + off[3j], y + off[3j+1], z + off[3j+2]); one outside
 * the grid is left out (not an error).  Terms are taken as for gathers:
 * neighbours in order j = 0..d-1, each with its read fields in ascending
 * id.  No index array is read.  Stencils must not write a field they read;
 * 1 <= d <= 32, |offsets| < the grid's extent. */
adha_status adha_section_create_stencil(const adha_struct *s, uint32_t n_read, const int32_t *read,
                                        uint32_t n_write, const int32_t *write, uint32_t nx, uint32_t ny,
                                        uint32_t nz, uint32_t d, const int32_t *offsets, adha_section **out);
/* A reduction section (section 3: the second K-Means section reduces all
 * the features over the points).  It reads n_read fields (F32, F64, I32 or
 * U32, at 4-byte aligned addresses in the layout it runs on) of every record
 * and, when key_field >= 0, the I32 key field, and adds
 * the values of the records whose key is k into row k of a table of
 * n_keys rows of n_read + 1 eight-byte cells, written to the device array
 * `out` (caller-owned, 256-byte aligned, out_cap >= n_keys*(n_read+1)*8):
 *   cell [k][j], j < n_read: the sum over those records of read field j
 *     (ascending id): an IEEE double for F32/F64 fields; a two's-complement
 *     int64 for I32 and U32 fields (exact);
 *   cell [k][n_read]: the number of those records (uint64).
 * Without a key every record has key 0 and n_keys must be 1.  Records whose
 * key is outside [0, n_keys) are left out and reported by adha_ctx_check.
 * Floating-point sums are compensated: each thread keeps its rounded sum
 * and the exact rounding errors, and partial sums are combined as
 * double-double numbers, in an order fixed by N, n_keys, n_read and the
 * device's CU count -- repeated runs give the same bits, and no
 * floating-point atomics are used.  The cell holds the double nearest the
 * double-double result.  For a cell with exact sum S and A = sum|x| over
 * its values, that result is within 2^-92 * A of S when n_keys <= 8 and
 * N <= 2^26 (more keys add at most 2^-105 * A per record of one workgroup),
 * so the cell is within 1 ulp of S correctly rounded whenever
 * A <= 2^38 * |S| in that range.  An exact zero sum is +0.0.  Values must be
 * finite, with partial sums below 2^1023 in magnitude.  Option
 * ADHA_OPT_REDUCE_COMPENSATED = 0 switches to plain double sums in the same
 * order (error up to (m-1) * 2^-53 * A for m values).
 * n_keys*(n_read+1) <= ADHA_MAX_REDUCE_CELLS.  The key may not be read.
 * Each run overwrites the whole table; `out` must not overlap the data. */
adha_status adha_section_create_reduce(const adha_struct *s, uint32_t n_read, const int32_t *read,
                                       int32_t key_field, uint32_t n_keys, void *out, uint64_t out_cap,
                                       adha_section **out_sec);
adha_status adha_section_destroy(adha_section *sec);
/* Runs the section in place on buf laid out by l.  idx (device, int32,
 * idx_count >= N*degree) is needed only for gather sections. */
adha_status adha_section_run(adha_ctx *ctx, const adha_section *sec, const adha_layout *l,
                             void *buf, uint64_t buf_cap, const int32_t *idx, uint64_t idx_count,
                             void *stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * as adha_section_run, but it allocates nothing.  A reduction's partial sums
 * (at most 16 MiB) live in a static device array of the library, one per
 * GPU, held until the process ends; pass 1 writes every partial pass 2
 * reads, so nothing has to start at zero.  All calls on one GPU share that
 * array: calls that overlap in time on one GPU (two streams, two threads)
 * race, so serialise them.  ERR_INVALID if a reduction would need more than
 * the array holds; other sections use no scratch. */
adha_status adha_section_run_static(adha_ctx *ctx, const adha_section *sec, const adha_layout *l,
                                    void *buf, uint64_t buf_cap, const int32_t *idx, uint64_t idx_count,
                                    void *stream);
/* Algorithmic bytes one run moves: N*(read + write bytes) for direct
 * sections and stencils (a stencil's neighbours are records of the same
 * arrays, so at the minimum each element is read once), N*(4*d + d*read +
 * write bytes) for gathers over an index array, N*(read + key bytes) for
 * reductions. */
adha_status adha_section_bytes(const adha_section *sec, uint64_t *out);
/* Effective HBM bytes one run moves under layout l, counted in 128-byte
 * access granules (the line a random access fetches, measured with
 * adha_probe_gather): a streamed group costs min(S_g, sum over touched
 * fields of max(e_f, 128/T)) per record; a gathered neighbour costs the
 * touched span of an interleaved group plus 127 bytes, else e_f + 127 per
 * field; a gather also reads 4*d index bytes.  This is the analytic cost
 * model's byte count (the unit of the gathers' transaction roofline). */
adha_status adha_section_effective_bytes(const adha_section *sec, const adha_layout *l, double *out);

/* ------------------------------------------------------------ host backend */
/* The same section on host memory with `threads` host threads (0: one per
 * core, at most 64), for plans that map sections to the CPU (section 2:
 * each section runs on the CPU or the GPU).  Results are identical to the
 * device kernels' (the same operations in the same order and rounding; a
 * reduction's double sums may differ in rounding order only).  idx is a
 * host array for gathers; a reduction writes its table to the host array
 * `table` (the device array given at creation is not touched).  *bad (may
 * be NULL) receives the number of out-of-range indices or keys. */
adha_status adha_host_section_run(const adha_section *sec, const adha_layout *l, void *buf, uint64_t buf_cap,
                                  const int32_t *idx, uint64_t idx_count, void *table, uint64_t table_cap,
                                  uint32_t threads, uint64_t *bad);
/* A remap between host buffers (padding zero-filled; out of place). */
adha_status adha_host_remap(const adha_layout *src_l, const void *src, uint64_t src_cap,
                            const adha_layout *dst_l, void *dst, uint64_t dst_cap, uint32_t threads);

/* ------------------------------------------------------------ programs */
adha_status adha_program_create(const adha_struct *s, uint32_t k, const adha_section *const *secs,
                                adha_program **out);
adha_status adha_program_destroy(adha_program *p);

/* Structured control flow (section 2: the sections form a structured
 * control-flow graph): the program's sections in a sequence with two-way
 * branches, as a token list -- a section index s >= 0 runs section s;
 * ADHA_TOK_IF opens a branch whose first part runs with probability
 * probs[i] (i counts IFs in order); ADHA_TOK_ELSE starts its second part
 * (optional); ADHA_TOK_END closes it.  Every section appears exactly once.
 * Plans of such a program minimise the expected cost over the branch
 * outcomes; the layout at each join is chosen too (a branch part that
 * ends in another layout is remapped there).  n_tokens = 0 restores the
 * plain sequence. */
#define ADHA_TOK_IF (-1)
#define ADHA_TOK_ELSE (-2)
#define ADHA_TOK_END (-3)
adha_status adha_program_set_flow(adha_program *p, uint32_t n_tokens, const int32_t *tokens, const double *probs);

/* Affinity weights (section 2, the ODS pass) of sections first..last:
 * w[a*F + b] for a != b.  Per loop iteration, fields touched at the same
 * record co-occur once: a direct section adds 1 to every pair of R u W; a
 * gather adds d to every pair of R and 1 to every pair of W. */
adha_status adha_affinity(const adha_program *p, uint32_t first, uint32_t last, uint64_t *w);
/* Greedy clustering (section 2, the ODS pass) of the merged sections
 * first..last under cap_bytes: edges by decreasing weight, ties by
 * (smaller id, larger id), join two clusters when their bytes fit.
 * Writes a layout (clusters interleaved with the given tile, every other
 * field on its own). */
adha_status adha_ods(const adha_program *p, uint32_t first, uint32_t last, uint32_t cap_bytes,
                     uint32_t tile, adha_layout **out);
/* Shortest path (section 2, the PDL pass) through the layered DAG of k
 * sections by C candidates: T[s*C + c] section costs, R[a*C + b] remap
 * costs (diagonal ignored, taken as 0), R0[c] start costs (NULL = 0).
 * Ties go to the smaller candidate index.  path[k] receives the choice. */
adha_status adha_pdl_solve(uint32_t k, uint32_t C, const double *T, const double *R,
                           const double *R0, uint32_t *path, double *cost);

/* The expected-cost shortest path of a structured program (tokens and
 * probs as for adha_program_set_flow) over k sections by C candidates with
 * the tables of adha_pdl_solve: node[k] per section, join[b] per branch,
 * *start the node the data starts in. */
adha_status adha_flow_solve(uint32_t k, uint32_t C, const double *T, const double *R, const double *R0,
                            uint32_t n_tokens, const int32_t *tokens, const double *probs, uint32_t *node,
                            uint32_t *join, uint32_t *start, double *cost);

/* ------------------------------------------------------------ planning */
typedef enum {
  ADHA_COST_MEASURED = 0, /* time every (section, candidate) on the device */
  ADHA_COST_ANALYTIC = 1, /* bytes moved / bandwidth, no device work */
  ADHA_COST_LEARNED = 2   /* the trained cost model; falls back to MEASURED */
} adha_cost_source;
typedef enum { ADHA_CAT_AOS_SOA = 0, ADHA_CAT_FULL = 1 } adha_catalogue;
/* FREE: data starts in the first chosen layout (and device) at no cost;
 * AOS: in AoS on the GPU; HOST_AOS: in AoS on the host (plans over both
 * devices only). */
typedef enum { ADHA_INIT_FREE = 0, ADHA_INIT_AOS = 1, ADHA_INIT_HOST_AOS = 2 } adha_init;
/* Where sections may run (section 2: the tuning profile holds CPU and GPU
 * times and the path picks a device per section). */
typedef enum { ADHA_DEVICES_GPU = 0, ADHA_DEVICES_GPU_HOST = 1 } adha_devices;

typedef struct {
  adha_cost_source cost;
  adha_catalogue catalogue;
  uint32_t cap_bytes; /* ODS structure capacity in bytes (default 128: one line) */
  adha_init init;     /* FREE: data starts in the first chosen layout at no cost */
  uint32_t reps;      /* measured costs: median of this many timed runs
                       * after a warm-up; with reps = 1 a section launch
                       * whose warm-up takes 2 ms or more is timed once */
  adha_devices devices; /* GPU only, or GPU and host */
  uint32_t pair_remaps; /* MEASURED, linear GPU programs: 1 (default) times the
                         * in-place remap of every ordered pair of candidates;
                         * 0 scales one measured whole-struct remap by the
                         * bytes each pair moves (as LEARNED does) */
  uint32_t verify_rounds; /* LEARNED, linear GPU programs: 0 (default) plans on
                           * the network's predictions alone; r > 0 then times
                           * the sections of the chosen path on the device,
                           * puts those times in the table and solves again,
                           * up to r rounds or until the chosen path is timed
                           * throughout (adha_plan_verified counts the timings) */
} adha_plan_opts;

adha_status adha_plan_opts_default(adha_plan_opts *o);
/* Builds the candidate catalogue (AoS, SoA, AoS tiled by 64, and the ODS
 * layout of every run of consecutive sections, interleaved and tiled),
 * fills the cost tables from the chosen source and solves the shortest
 * path.  Measured and learned costs use device scratch the call allocates
 * and frees; gather sections are timed with idx (device, N*d entries) when
 * given, else with uniformly random neighbours.  A section is timed once per
 * distinct arrangement of the groups holding its fields: candidates that
 * differ only in groups the section does not touch share that time.
 * Remap costs (section 2:
 * weighed by the fields two layouts have in common): for linear GPU
 * programs a remap a -> b moves only the fields whose group (fields and
 * tile) differs, as adha_run_placed runs it -- MEASURED times every ordered
 * pair that way, ANALYTIC charges 4 us + 2*N*(their bytes) / 5.6 TB/s,
 * LEARNED (and MEASURED with pair_remaps = 0) scales one measured
 * whole-struct remap by the bytes each pair moves; for structured programs and plans over both devices every pair of
 * different layouts costs one whole-struct remap (measured, or analytic
 * with all N*S bytes), as their executors remap between two buffers.
 * Returns WARN_FALLBACK when LEARNED had no model. */
adha_status adha_plan_create(adha_ctx *ctx, const adha_program *p, const adha_plan_opts *o,
                             const int32_t *idx, uint64_t idx_count, void *stream,
                             adha_plan **out);
/* The same linear GPU plan solved again, with its candidates and cost
 * tables, for data that starts FREE (in the first chosen layout, at no
 * cost) or in AoS (INIT_AOS: the entry remap from AoS is charged and run).
 * No device work.  ERR_UNSUPPORTED for structured programs and plans over
 * both devices. */
adha_status adha_plan_with_init(const adha_plan *pl, adha_init init, adha_plan **out);
/* A plan that keeps one layout for every section (the all-AoS / all-SoA
 * baselines). */
adha_status adha_plan_uniform(const adha_program *p, const adha_layout *l, adha_plan **out);
/* A plan given section by section: layouts[k] and devices[k] (0 the GPU,
 * 1 the host; NULL = all on the GPU).  Its cost tables are zero. */
adha_status adha_plan_explicit(const adha_program *p, const adha_layout *const *layouts, const int32_t *devices,
                               adha_plan **out);
/* Candidate layout at the join of branch i (structured programs). */
adha_status adha_plan_join(const adha_plan *pl, uint32_t i, uint32_t *candidate);
/* Runs a structured program (any plan of it, GPU sections only) along the
 * branch outcomes taken[i] (1: the first part of branch i, 0: the second),
 * n_taken >= the number of branches; otherwise as adha_run. */
adha_status adha_run_flow(adha_ctx *ctx, const adha_plan *pl, const adha_layout *in_layout, void *buf_a,
                          void *buf_b, uint64_t buf_cap, const int32_t *idx, uint64_t idx_count,
                          const uint8_t *taken, uint32_t n_taken, void *stream, const adha_layout **out_layout,
                          int32_t *out_in_b);
/* Device of section s's choice: 0 the GPU, 1 the host. */
adha_status adha_plan_device(const adha_plan *pl, uint32_t s, int32_t *device);
/* The shortest-path graph: M nodes (C for GPU plans; 2C over both devices,
 * node m = (device m / C, candidate m % C)); T[k*M] section costs and
 * R[M*M] move costs in microseconds.  Over both devices a move between
 * devices costs one transfer of the struct each way (measured with pinned
 * host memory, or analytic at 50 GB/s) plus, when the layout changes, the
 * GPU remap (done on the GPU side); a host remap costs the measured host
 * remap.  Host section costs are measured with the context's host threads
 * (median of reps) or analytic (bytes at 40 GB/s plus 30 us). */
adha_status adha_plan_nodes(const adha_plan *pl, uint32_t *M);
adha_status adha_plan_node_tables(const adha_plan *pl, double *T, double *R);
adha_status adha_plan_destroy(adha_plan *pl);
adha_status adha_plan_n_candidates(const adha_plan *pl, uint32_t *out);
/* Candidate c's layout; the plan owns it. */
adha_status adha_plan_candidate(const adha_plan *pl, uint32_t c, const adha_layout **out);
adha_status adha_plan_choice(const adha_plan *pl, uint32_t s, uint32_t *candidate);
/* Predicted program cost in microseconds under the plan's cost tables. */
adha_status adha_plan_cost(const adha_plan *pl, double *us);
/* Copies the cost tables (T: k*C, R: C*C, microseconds); either may be NULL. */
adha_status adha_plan_tables(const adha_plan *pl, double *T, double *R);
/* Seconds spent building the plan (catalogue, costs, path). */
adha_status adha_plan_time(const adha_plan *pl, double *seconds);
/* (section, candidate) entries a learned plan timed to verify its path
 * (opts.verify_rounds); 0 for other plans. */
adha_status adha_plan_verified(const adha_plan *pl, uint32_t *entries);

/* Runs the program under the plan with two buffers.  The data starts in
 * buf_a laid out by in_layout (under INIT_FREE pass the plan's first
 * layout, or any layout, in which case a remap is made first).  Between
 * sections with different layouts the whole struct is remapped into the
 * other buffer (so a linear plan priced for adha_run_placed may take longer
 * than predicted).  *out_layout (owned by the plan or equal to in_layout)
 * and *out_in_b tell where it ends. */
adha_status adha_run(adha_ctx *ctx, const adha_plan *pl, const adha_layout *in_layout,
                     void *buf_a, void *buf_b, uint64_t buf_cap, const int32_t *idx,
                     uint64_t idx_count, void *stream, const adha_layout **out_layout,
                     int32_t *out_in_b);
/* Placed execution (section 2: remap edges weighed by the fields two
 * layouts have in common).  The program runs in one device buffer, the
 * arena: between two sections the groups both layouts hold (same fields
 * and tile) stay where they are and only the others are moved
 * (adha_remap_in_place), into free space of the arena.  The placement is
 * fixed when the plan is made: *bytes is the arena size it needs, *start
 * the layout the data must be in before the run (the plan's first layout,
 * or AoS under INIT_AOS, at its canonical bases from the arena's start),
 * *end the placed layout the data ends in (both owned by the plan; remap
 * *end to any layout to read the result).  Plans made by adha_plan_create
 * for linear GPU programs are priced for this executor: their remap costs
 * are per pair of layouts.  ERR_UNSUPPORTED for structured programs and
 * plans over both devices. */
adha_status adha_plan_arena(const adha_plan *pl, uint64_t *bytes, const adha_layout **start,
                            const adha_layout **end);
/* Placed layout i of the plan, i in [0, k]: i = 0 the start layout, i =
 * s + 1 the layout section s runs in.  Owned by the plan. */
adha_status adha_plan_placed(const adha_plan *pl, uint32_t i, const adha_layout **out);
/* Runs the plan placed in `arena` (device, 256-byte aligned, arena_cap >=
 * the plan's arena bytes), data starting in the plan's start layout.  idx
 * as for adha_run.  Everything is validated before the first launch. */
adha_status adha_run_placed(adha_ctx *ctx, const adha_plan *pl, void *arena, uint64_t arena_cap,
                            const int32_t *idx, uint64_t idx_count, void *stream);

/* Runs a plan whose sections may be mapped to the host (the same as
 * adha_run for GPU plans, which reject host sections).  The data starts in
 * dev_a (in_device 0) or host_a (in_device 1), laid out by in_layout.  A
 * GPU section runs on `stream` in the device buffers, a host section with
 * the context's host threads in the host buffers (after the stream has
 * drained).  A move between devices copies the struct over; when it also
 * changes the layout the remap happens on the GPU side.  Host buffers
 * should be pinned for full copy speed.  Gathers need idx_dev (device,
 * 256-byte aligned) and/or idx_host (host) as their sections' devices
 * require, each holding idx_count >= N*d entries.  A reduction on the host
 * copies its table to the device array given at creation.  The call
 * returns once host work is done; GPU work may still be in flight.
 * *out_device (0/1) and *out_in_b tell where the data ends. */
adha_status adha_run_hetero(adha_ctx *ctx, const adha_plan *pl, const adha_layout *in_layout, int32_t in_device,
                            void *dev_a, void *dev_b, void *host_a, void *host_b, uint64_t buf_cap,
                            const int32_t *idx_dev, const int32_t *idx_host, uint64_t idx_count, void *stream,
                            const adha_layout **out_layout, int32_t *out_device, int32_t *out_in_b);

/* ------------------------------------------------------------ probes */
/* Bandwidth ceilings of the device, with plain kernels of the library:
 * kind 0 reads `bytes` of a, kind 1 writes `bytes` of b, kind 2 copies a to
 * b, all as 16-byte accesses over a persistent grid.  *us is the best, over
 * a sweep of 48 forms (1, 2, 4 or 8 chunks in flight per thread; ordinary
 * or streaming accesses; 4, 8 or 16 workgroups per CU; the grid striding
 * over the buffer or each workgroup streaming a contiguous share), of the
 * median of reps timed launches after one warm-up.  Buffers are
 * device, 256-byte aligned, `bytes` each (a multiple of 16; b is the read
 * probe's sink and stays unwritten in practice); a and b may not overlap
 * for a copy.  GB/s = bytes (read, write) or 2*bytes (copy) / us / 1e3. */
adha_status adha_probe_stream(adha_ctx *ctx, uint32_t kind, void *a, void *b, uint64_t bytes, uint32_t reps,
                              void *stream, double *us);
/* Random-access probe (the access of a gather's neighbour field): lane i
 * loads load_bytes (4, 8, 16, 32, 64 or 128; above 16 as 16-byte loads)
 * at buf + idx[i] * stride and writes one
 * 4-byte word to out[i], for i < n (n <= 2^28).  Every index is checked on
 * the host to name a record inside buf (idx[i] < buf_bytes / stride) before
 * the launch.  *us as for adha_probe_stream.  n / us is the random-access
 * rate; with the HBM bytes a counter run reports it gives the bytes one
 * random access fetches. */
adha_status adha_probe_gather(adha_ctx *ctx, const void *buf, uint64_t buf_bytes, uint64_t stride,
                              uint32_t load_bytes, const int32_t *idx, uint64_t n, void *out, uint32_t reps,
                              void *stream, double *us);

/* ------------------------------------------------------------ cost model */
#define ADHA_N_FEATURES 16
/* Feature vector of (section, layout) for the learned cost model. */
adha_status adha_features(const adha_section *sec, const adha_layout *l, float *out16);

/* Network: 16 -> 64 -> 64 -> 64 -> 1 (ReLU), fp32, predicting ln(time in
 * microseconds).  Parameters are one fp32 array: W0[64][16], b0[64],
 * W1[64][64], b1[64], W2[64][64], b2[64], W3[1][64], b3[1]. */
#define ADHA_MLP_PARAMS (64 * 16 + 64 + 64 * 64 + 64 + 64 * 64 + 64 + 64 + 1)
/* Device kernels of the network, on caller-owned device buffers:
 * forward: x [B][16] -> y [B]; backward: gradient of mean((y - t)^2) into
 * grad [ADHA_MLP_PARAMS] (overwritten) and, if loss != NULL, the loss
 * (device float); adam: one Adam step (lr, b1, b2, eps, step count t >= 1)
 * on params with moments m, v. */
adha_status adha_mlp_forward(adha_ctx *ctx, const float *params, const float *x, uint32_t batch,
                             float *y, void *stream);
adha_status adha_mlp_backward(adha_ctx *ctx, const float *params, const float *x,
                              const float *target, uint32_t batch, float *grad, float *loss,
                              void *stream);
adha_status adha_mlp_adam(adha_ctx *ctx, float *params, const float *grad, float *m, float *v,
                          float lr, float b1, float b2, float eps, uint32_t t, void *stream);

typedef struct {
  uint32_t n_samples;  /* sections to generate and time */
  uint32_t epochs;
  uint32_t batch;
  float lr;            /* Adam's initial step size; it decays along a half cosine to lr / 20 */
  uint64_t seed;
  int32_t min_log2_n, max_log2_n; /* record counts of generated sections */
  uint32_t reps;       /* timing: median of reps */
  uint32_t progress_every; /* >0: one line on stderr per that many timed sections */
  uint32_t ensemble;   /* networks trained on the same timings from different
                        * initial weights (1..16, default 1); the model
                        * predicts with their mean */
} adha_train_opts;
typedef struct {
  double gen_seconds, train_seconds;
  double train_loss, val_loss;
  double val_mape;     /* mean absolute percentage error of predicted time */
  uint32_t n_train, n_val;
} adha_train_report;
adha_status adha_train_opts_default(adha_train_opts *o);
/* Generates sections and layouts, times them on the device, trains the
 * network(s) with the kernels above and keeps the model in the context.
 * The model predicts ln(time / analytic estimate) of a (section, layout)
 * as the mean over its networks; the planner uses the analytic estimate
 * times e^prediction.  val_loss and val_mape are those of that mean. */
adha_status adha_costmodel_train(adha_ctx *ctx, const adha_train_opts *o, adha_train_report *rep);
adha_status adha_costmodel_save(const adha_ctx *ctx, const char *path);
/* Model files: "ADHAMLP3", the network count, the parameter count per
 * network, the parameters, an FNV-1a checksum.  ERR_IO on a missing, short
 * or corrupt file (checksum); the context then keeps no model. */
adha_status adha_costmodel_load(adha_ctx *ctx, const char *path);
/* Predicted time (microseconds) of sec under l with the loaded model. */
adha_status adha_costmodel_predict(adha_ctx *ctx, const adha_section *sec, const adha_layout *l,
                                   double *us);

#ifdef __cplusplus
}
#endif
#endif /* ADHA_H */
