/*
 * smmo.h - C ABI of libsmmo, Single-Method Multiple-Objects execution on
 * AMD Instinct MI355X (gfx950).
 *
 * Programming model (Springer, "Memory-Efficient Object-Oriented Programming
 * on GPUs", Ch.3 sec.3.2.1 "Definition and Runtime Semantics" and Ch.5
 * sec.5.1.1 "Programming Interface"): objects of user-defined classes live on
 * a device heap; parallel_do runs one method on every object of a class that
 * exists when the operation starts; methods may create objects of any class
 * (the new objects are not visited by the running operation) and may delete
 * their own object as their last action, or objects of other classes.
 *
 * Storage (Ch.5 sec.5.2 "Architecture Overview"): the heap is divided into M
 * blocks of equal size.  A block holds up to 64 objects of one class in
 * structure-of-arrays layout: one contiguous 64-entry array per field (per
 * inner-array element), so the 64 lanes of a wavefront touch one contiguous
 * run of memory per field.  Every class gets capacity 64 (the thesis gives
 * capacity 64 to the smallest class, sec.5.2.2 "Block Capacity"; a wavefront
 * is 64 lanes wide on CDNA).  Block states and free space are indexed by
 * hierarchical bitmaps (sec.5.3.1).
 *
 * Conventions for every call:
 *   - The return value is an smmo_status: SMMO_OK or a negative error code.
 *     smmo_last_error() gives a text description of the last error raised on
 *     the calling host thread.
 *   - Argument errors are detected on the host before anything is enqueued;
 *     nothing is enqueued when a call fails.
 *   - Device-side errors (heap exhausted during an allocation, a handle that
 *     does not name a live object of the class, a retry loop that exceeded
 *     its bound) set an error word on the device.  Every later kernel on the
 *     heap sees the word and does nothing; the next smmo_sync() or
 *     smmo_heap_stats() returns it (SMMO_ENOMEM or SMMO_EDEVICE).
 *   - "stream" is a hipStream_t (NULL = the default stream).  Calls enqueue
 *     work and return without waiting, except smmo_sync(), smmo_heap_stats(),
 *     smmo_check_invariants() and smmo_heap_free(), which wait.  All calls on
 *     one heap must be ordered on the host and on the device (one stream, or
 *     streams joined by events); two calls on one heap that run at the same
 *     time on the device race, with one exception: two parallel_do calls on
 *     classes of different families may run at the same time (the device
 *     allocator is safe under concurrency) if neither deletes objects of
 *     the class the other walks, a class that gets new objects from one is
 *     walked by the other only through a snapshot (smmo_snapshot), and
 *     the methods' reads and writes of fields do not conflict.
 *   - Device pointers are addresses in device memory of the GPU the heap is
 *     on.  The caller owns every buffer it passes and keeps it alive until the
 *     work that uses it has completed.  libsmmo allocates no device memory:
 *     the heap and all of its internal arrays are carved out of the buffer
 *     given to smmo_alloc_heap().
 *   - Handles are 32-bit: (block index << 6) | slot.  SMMO_NULL names no
 *     object.  Handles of live objects are < 2^31, so the top bit is free for
 *     the caller to use as a flag in handle-valued fields.
 */
#ifndef SMMO_H
#define SMMO_H

#include <stddef.h>
#include <stdint.h>

#include "smmo_methods.h"   /* argument structs of the compiled-in methods */

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t smmo_status;
#define SMMO_OK 0
#define SMMO_EINVAL (-1)        /* bad argument                                */
#define SMMO_ENOMEM (-2)        /* heap exhausted / buffer too small           */
#define SMMO_ESTATE (-3)        /* call not allowed in the current state       */
#define SMMO_EHIP (-4)          /* a HIP runtime call failed                   */
#define SMMO_EDEVICE (-5)       /* device-side error (see smmo_sync)           */
#define SMMO_EUNSUPPORTED (-6)  /* feature or method not available             */

typedef uint32_t smmo_handle;
#define SMMO_NULL 0xFFFFFFFFu

typedef void *smmo_stream;      /* a hipStream_t */

/* field element types */
#define SMMO_U8 1
#define SMMO_I32 2
#define SMMO_U32 3
#define SMMO_F32 4
#define SMMO_HANDLE 5           /* uint32 handle (or handle with flag bit 31) */

#define SMMO_MAX_CLASSES 16
#define SMMO_MAX_FIELDS 32      /* per class, counting every inner-array element */
#define SMMO_BLOCK_CAPACITY 64

typedef struct smmo_schema smmo_schema;
typedef struct smmo_heap smmo_heap;

/* One field of a class.  count > 1 declares an inner array of `count`
 * elements stored as `count` separate 64-entry SOA arrays ("SOA with full
 * inlining" of inner arrays, Ch.4 sec.4.3.1), so that element q of 64
 * objects is one contiguous run. */
typedef struct {
    const char *name;           /* unique within the class, <= 31 chars */
    int32_t dtype;              /* SMMO_U8 .. SMMO_HANDLE */
    uint32_t count;             /* inner-array length, >= 1 */
} smmo_field_desc;

/* Heap configuration (smmo_config_default() fills the defaults). */
typedef struct {
    uint32_t lookup_retries;    /* active-block lookups before the slow path
                                   (Ch.5 sec.5.3.2 "Lookup Retry"); default 5 */
    uint32_t rotation;          /* 1: rotate bitmap containers before
                                   find-first-set ("Bitmap Rotation"); default 1 */
    uint32_t coalescing;        /* 1: one leader lane allocates for all lanes of a
                                   wavefront ("Allocation Request Coalescing");
                                   0: every lane allocates on its own; default 1 */
    uint32_t bulk_ordered;      /* 1: smmo_parallel_new claims free blocks in
                                   ascending order and fills them densely;
                                   0: every object goes through the device
                                   allocator; default 1 */
    uint32_t spin_limit;        /* bound on every retry loop; exceeding it sets
                                   SMMO_EDEVICE instead of hanging; default 1<<20 */
    uint32_t grid_waves;        /* wavefronts per method launch (0 = automatic) */
    uint32_t block_group;       /* blocks a wavefront loads together before it
                                   computes, in the methods that support it
                                   (1, 2 or 4; 0 = each method's default) */
    uint32_t sparse_packing;    /* methods that can run packed do-alls (the
                                   classes that births and deaths fragment): a
                                   block with at most 32 live objects is sparse,
                                   and two sparse blocks share a wavefront.
                                   0: never pack (default; every block gets a
                                   wavefront of its own);
                                   1: pack when the class may have more blocks
                                   than the launch has wavefronts, so that
                                   packing shortens the wavefronts' walks;
                                   2: always pack.  Modes 1 and 2 make the
                                   enumeration read every listed block's bitmap
                                   to build the packing plan. */
    uint32_t streaming_loads;   /* spring.force and spring.node_update: load
                                   the fields each do-all reads once (not the
                                   gathered ones) with a non-temporal hint.
                                   0: when the node and spring blocks exceed
                                   the 256 MB MALL (default; a step's blocks
                                   that fit in it are reused by the next step);
                                   1: never; 2: always.  Same results. */
    uint32_t reserved[7];
} smmo_config;

typedef struct {
    uint64_t live_objects[SMMO_MAX_CLASSES];
    uint64_t blocks[SMMO_MAX_CLASSES];       /* allocated blocks per class */
    uint64_t free_blocks;
    uint64_t total_blocks;                   /* M */
    double fragmentation;                    /* unused slots / slots of allocated
                                                blocks (Ch.5 sec.5.6.3, "F") */
    int32_t device_error;                    /* SMMO_OK, SMMO_ENOMEM or SMMO_EDEVICE */
    uint32_t block_bytes;
    uint64_t slow_paths;                     /* blocks initialized by device new */
    uint64_t alloc_retries;                  /* failed reservations, all retried */
    uint64_t device_news;                    /* objects created by device allocation
                                                (methods, non-ordered parallel_new) */
    uint64_t device_deletes;                 /* objects released by device
                                                deallocation (methods, smmo_destroy) */
    uint64_t bitmap_spins;                   /* extra rounds of converged bitmap
                                                switches (a switch found its bit
                                                not yet in the expected state) */
    uint64_t lookups;                        /* active-block and free-block searches */
} smmo_stats;

typedef struct {
    uint64_t hierarchy_violations;   /* summary bit != OR of its container  */
    uint64_t state_violations;       /* block not exactly one of free / allocated[type] */
    uint64_t active_violations;      /* active[C] set <=> allocated[C] and not full */
    uint64_t type_violations;        /* allocated[C] set but block type != C */
    uint64_t empty_allocated;        /* allocated blocks with no object */
} smmo_invariants;

/* A field initializer for smmo_parallel_new: `values` is a device pointer to
 * n * count elements of the field's type, object i's elements at
 * [i*count, (i+1)*count).  Fields without an initializer are zero-filled. */
typedef struct {
    uint32_t field_id;
    const void *values;
} smmo_field_init;

/* ---- configuration and schema ------------------------------------------ */

void smmo_config_default(smmo_config *cfg);

/* Creates an empty schema.  *out receives it; free with smmo_schema_free(). */
smmo_status smmo_schema_create(smmo_schema **out);
smmo_status smmo_schema_free(smmo_schema *s);

/* Declares a class (the thesis declares classes and field types at compile
 * time, Ch.5 sec.5.1.1 "Data Layout DSL"; here at run time).  Fields are laid
 * out in the given order.  *class_id receives 0, 1, ... in definition order.
 * Fails with SMMO_ESTATE once a heap was created from the schema, SMMO_EINVAL
 * for duplicate or empty names, bad types, count 0, or more than
 * SMMO_MAX_FIELDS arrays, SMMO_ENOMEM for more than SMMO_MAX_CLASSES classes. */
smmo_status smmo_define_class(smmo_schema *s, const char *name,
                              const smmo_field_desc *fields, uint32_t nfields,
                              uint32_t *class_id);

/* Declares a class that derives from `parent` (single inheritance, thesis
 * Ch.5 sec.5.1.1 "Class Inheritance"; the block's data segment holds the
 * inherited field arrays first, then the new ones, sec.5.2.1 "Block
 * Structure").  Its fields are the parent's, at the same offsets inside a
 * block and with the same field ids, followed by `fields` (nfields may be 0;
 * fields may then be NULL).  So a method bound to the fields of a class runs
 * unchanged on the blocks of every descendant.  parent = SMMO_NO_PARENT
 * declares a root class.  flags: SMMO_CLASS_ABSTRACT for a class without
 * objects of its own (the thesis's kIsAbstract): smmo_parallel_new refuses it
 * and no method allocates it.
 * A do-all (smmo_parallel_do) on a class runs the method on the objects of
 * the class and of all its descendants: one kernel per concrete class of that
 * family, in class-id order, each class enumerated just before its kernel
 * (the thesis launches a separate kernel per type to avoid divergence).
 * Errors as smmo_define_class; SMMO_EINVAL for a bad parent or flags. */
#define SMMO_NO_PARENT 0xFFFFFFFFu
#define SMMO_CLASS_ABSTRACT 1u
smmo_status smmo_define_subclass(smmo_schema *s, const char *name, uint32_t parent, uint32_t flags,
                                 const smmo_field_desc *fields, uint32_t nfields,
                                 uint32_t *class_id);

/* *out = 1 if class `cls` is `ancestor` or derives from it, else 0 (the
 * relation behind cast<T>, Ch.5 sec.5.1.1). */
smmo_status smmo_class_is_a(const smmo_schema *s, uint32_t cls, uint32_t ancestor, uint32_t *out);

/* Looks up a field of a class by name; *field_id is its index in the
 * class's field list (inherited fields first). */
smmo_status smmo_field_id(const smmo_schema *s, uint32_t class_id, const char *name,
                          uint32_t *field_id);

/* Bytes of one block (the largest class's 64-object data segment), and the
 * device buffer size smmo_alloc_heap() needs for a heap of `blocks` blocks. */
smmo_status smmo_block_bytes(const smmo_schema *s, uint32_t *block_bytes);
smmo_status smmo_heap_bytes(const smmo_schema *s, uint64_t blocks, uint64_t *bytes);

/* ---- heap -------------------------------------------------------------- */

/* A caller-supplied device allocator, for heaps created without a buffer:
 * alloc(bytes, ctx) returns `bytes` bytes of device memory on the current
 * device, 256-byte aligned, or NULL; release(ptr, bytes, ctx) gives back
 * what alloc returned.  Both are called on the thread that creates or frees
 * the heap, never from a kernel or a stream callback. */
typedef struct {
    void *(*alloc)(size_t bytes, void *ctx);
    void (*release)(void *ptr, size_t bytes, void *ctx);
    void *ctx;
} smmo_allocator;

/* Sets the allocator that smmo_alloc_heap() uses when dev_buf is NULL
 * (process-wide; NULL unsets it).  A heap keeps the allocator it was created
 * with and releases its buffer through it in smmo_heap_free().  SMMO_EINVAL
 * if alloc or release is NULL. */
smmo_status smmo_set_allocator(const smmo_allocator *a);

/* Creates a heap in the caller's device buffer `dev_buf` of `bytes` bytes
 * (256-byte aligned), or, with dev_buf NULL, in `bytes` bytes taken from the
 * allocator set by smmo_set_allocator() (SMMO_EINVAL if none is set,
 * SMMO_ENOMEM if it returns NULL).  M, the number of blocks, is the largest
 * count whose arrays and blocks fit; at most 2^25 - 2.  Enqueues the
 * initialization (all blocks free, Ch.5 sec.5.2.4 "Block Bitmaps") on
 * `stream`.  The schema is frozen.  cfg may be NULL for the defaults.  A
 * caller's buffer must stay allocated until smmo_heap_free().  SMMO_ENOMEM if
 * not even one block fits. */
smmo_status smmo_alloc_heap(smmo_schema *s, void *dev_buf, size_t bytes,
                            const smmo_config *cfg, smmo_stream stream, smmo_heap **out);

/* Waits for the heap's work and releases host-side state, and the buffer if
 * the heap took it from an allocator (a caller's dev_buf stays the
 * caller's). */
smmo_status smmo_heap_free(smmo_heap *h);

/* ---- SMMO operations ---------------------------------------------------- */

/* parallel_new (Ch.5 sec.5.1.1): creates n objects of class `class_id`.
 * Object i takes its field values from the initializers (element i), other
 * fields are zero.  If out_handles (device, n entries) is not NULL,
 * out_handles[i] receives object i's handle.  n = 0 is a no-op.  The host
 * rejects n > 64 * M with SMMO_ENOMEM; if the free blocks do not suffice the
 * device sets SMMO_ENOMEM (bulk_ordered: nothing is created; otherwise the
 * objects that found room exist and the others' handles are SMMO_NULL). */
smmo_status smmo_parallel_new(smmo_heap *h, uint32_t class_id, uint32_t n,
                              const smmo_field_init *init, uint32_t ninit,
                              uint32_t *out_handles, smmo_stream stream);

/* parallel_do (Ch.3 sec.3.2.1; Ch.5 sec.5.2.7): runs method `method_id` once
 * on every object of class `class_id` alive when the launch starts.  `args`
 * points to the method's argument struct (host memory, copied before return;
 * smmo_methods.h), args_bytes its size.  The method must accept the class:
 * each method names the fields it needs (by name and type) and fails with
 * SMMO_EINVAL if the class lacks one. */
smmo_status smmo_parallel_do(smmo_heap *h, uint32_t class_id, uint32_t method_id,
                             const void *args, size_t args_bytes, smmo_stream stream);

/* Takes the iteration snapshot of class `class_id` and its concrete
 * descendants now, in `stream` order, for the next parallel_do on the class
 * (the enumeration of Ch.5 sec.5.2.7 with its copy of the allocation
 * bitmaps, moved ahead of the launch).  That parallel_do runs the method on
 * the objects alive at the snapshot, enumerates nothing, and may run on
 * another stream while other work creates objects of the class: objects
 * created after the snapshot are neither visited nor read.  Between the
 * snapshot and that parallel_do, device code may not delete objects of the
 * class (a do-all on another class that does breaks the snapshot; nothing
 * checks this).  smmo_destroy, smmo_gather_soa or smmo_defragment of the
 * class in between, or any other enumeration of it, drops the snapshot: the
 * parallel_do then takes its own at its start.  Errors as
 * smmo_parallel_do's: SMMO_EINVAL for a bad heap or class. */
smmo_status smmo_snapshot(smmo_heap *h, uint32_t class_id, smmo_stream stream);

/* destroy (Ch.5 sec.5.1.1; deallocation as in sec.5.2.6 and sec.5.4): deletes
 * the n objects whose handles are in the device array `handles`.  Each must
 * be a live object of class `class_id` and appear once; a handle that is not
 * sets SMMO_EDEVICE and is skipped.  Empty blocks return to the free state. */
smmo_status smmo_destroy(smmo_heap *h, uint32_t class_id, const uint32_t *handles,
                         uint32_t n, smmo_stream stream);

/* Copies fields of all live objects of a class into dense device arrays.
 * out_ptrs[j] (host array of nfields device pointers) receives field
 * field_ids[j]: capacity * count elements of the field's type.  out_handles
 * (device, may be NULL) receives the handles.  *out_count (device uint32)
 * receives the number of live objects; objects beyond `capacity` are not
 * written.  The order is unspecified (block by block). */
smmo_status smmo_gather_soa(smmo_heap *h, uint32_t class_id, const uint32_t *field_ids,
                            uint32_t nfields, void *const *out_ptrs, uint32_t *out_handles,
                            uint32_t capacity, uint32_t *out_count, smmo_stream stream);

/* A caller-owned device array of handles that smmo_defragment rewrites
 * together with the heap's own HANDLE fields (bit 31 of each entry is kept). */
typedef struct {
    uint32_t *handles;
    uint64_t count;
} smmo_handle_array;

/* The memory coalescing experiment (Ch.2, "Memory coalescing experiment")
 * on n floats at device pointer `data` (caller-owned): every element is read
 * and written once (x += 8) by a grid-stride loop over `grid` work-groups of
 * 256 threads (0 = 2048); the lanes of a wavefront touch C arrays of n/C
 * elements each (C = 1, 2, 4, .., 64; 1 = fully coalesced).  n must be a
 * multiple of 64 * C.  Asynchronous on `stream`; the caller times it.  A
 * measurement of the attainable bandwidth, not part of the object model. */
smmo_status smmo_coalescing_probe(float *data, uint64_t n, uint32_t C, uint32_t grid, smmo_stream stream);

/* Memory defragmentation of class `class_id` (CompactGpu, Ch.6): blocks that
 * are at most n/(n+1) full (n = 1..8, the defragmentation factor) are
 * candidates; in a pass, the first floor(d/(n+1)) of the d candidates are
 * source blocks, each merged into n other candidates, and become free.
 * Every live HANDLE field of every class, and every entry of the `next`
 * external arrays, that names a moved object is rewritten to its new handle
 * (bit 31 is kept; SMMO_NULL entries are skipped).  Passes repeat until at
 * most k1 candidates remain, fewer than n + 1 do, or max_passes ran.
 * Stop-the-world: nothing else may run on the heap meanwhile; objects keep
 * their field values but not their handles.  Handles held anywhere else go
 * stale.  Synchronizes (reads the candidate count once per pass).
 * out_passes and out_moved (host, may be NULL) receive the number of passes
 * and of moved objects. */
smmo_status smmo_defragment(smmo_heap *h, uint32_t class_id, uint32_t n, uint32_t k1, uint32_t max_passes,
                            const smmo_handle_array *ext, uint32_t next, smmo_stream stream,
                            uint32_t *out_passes, uint64_t *out_moved);

/* The removal of disconnected nodes (Ch.7 "structure": a breadth-first
 * search from the anchor nodes over the springs, then every node it does not
 * reach, and every spring of such a node, is deleted) as one call: the
 * do-alls bfs_init, bfs_visit (until a pass finds the frontier empty),
 * bfs_mark and bfs_delete with the same results (distances, deletions), the
 * frontier kept as a queue instead of found by a pass over every node, and
 * the visited set as a bitmap in the work-group's LDS.
 *   h, args   the heap and the structure classes (args->nodebase_class is the
 *             family searched, args->anchor_class its start nodes,
 *             args->bfs_options 0 or SMMO_BFS_* bits; distance, dt and flag
 *             are not used)
 *   work      device buffer of work_words uint32 words owned by the caller,
 *             at least 64 + C + M + C / 32 rounded up to a multiple of 4, plus
 *             4 C, where C = 64 B_n, B_n = the blocks the node classes may
 *             hold and M = the heap's blocks (B_n <= M, so 68 + 324 M always
 *             suffices); its contents on entry do not matter and on return are
 *             unspecified
 *   levels    device word: receives the number of visit passes the
 *             level-by-level form runs (the non-empty levels plus the one that
 *             finds the frontier empty), 0 if the heap has failed
 * Asynchronous on `stream`; SMMO_EINVAL (nothing enqueued) for NULL
 * pointers, bad classes, unknown bfs_options bits or a workspace too small;
 * device errors as for smmo_parallel_do. */
smmo_status smmo_structure_remove_disconnected(smmo_heap *h, const smmo_structure_args *args, uint32_t *work,
                                               uint64_t work_words, uint32_t *levels, smmo_stream stream);

/* smmo_structure_remove_disconnected without a workspace, for callers that
 * cannot allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid allocation): the same kernels and results, the
 * workspace being a device array of the library (about 21 MB on each GPU it
 * runs on, held until the process ends).  Allocates nothing.  The heap's
 * device must be the current device.  SMMO_EINVAL for a heap of more than
 * 16,384 blocks (pass a workspace to smmo_structure_remove_disconnected
 * instead), NULL pointers or bad classes.  All calls on one GPU share the
 * array: calls that overlap on one GPU (other streams, other threads, other
 * heaps) race and must be ordered by the caller. */
smmo_status smmo_structure_remove_disconnected_noalloc(smmo_heap *h, const smmo_structure_args *args,
                                                       uint32_t *levels, smmo_stream stream);

/* ---- synchronization, statistics, diagnostics --------------------------- */

/* Waits for all work enqueued on the heap and returns the device error word
 * (SMMO_OK, SMMO_ENOMEM or SMMO_EDEVICE). */
smmo_status smmo_sync(smmo_heap *h);

/* Waits, then fills *st (live objects and blocks per class, fragmentation,
 * the device error word).  Returns SMMO_OK even if device_error is set. */
smmo_status smmo_heap_stats(smmo_heap *h, smmo_stats *st);

/* Waits, then checks the block-state invariants that hold whenever no kernel
 * runs on the heap: bitmap hierarchy consistency (Ch.5 sec.5.4.5 "container
 * consistency"), free XOR allocated, active <=> allocated and not full. */
smmo_status smmo_check_invariants(smmo_heap *h, smmo_invariants *inv);

/* Resets the device error word (after the caller has handled it). */
smmo_status smmo_clear_error(smmo_heap *h, smmo_stream stream);

/* Number of blocks M and block size of a heap. */
smmo_status smmo_heap_info(const smmo_heap *h, uint64_t *blocks, uint32_t *block_bytes);

/* Launch shape of `method_id` on class `class_id` for this heap (the
 * autotuner's knobs): work-group size wg_threads (64, 128, 256, 512 or 1024;
 * 0 = default 256), grid_waves wavefronts in total (0 = default, 64 per CU)
 * and group, the number of blocks (1, 2 or 4; 0 = default) a wavefront loads
 * together before it computes on them, in the methods that support it
 * (spring.force, spring.node_update).  Each wavefront takes `group`
 * consecutive entries of the class's block list per iteration and skips
 * grid_waves * group entries, so blocks per wavefront = ceil(blocks of the
 * class / grid_waves).  Methods with a fixed shape (nbody.force) ignore it.
 * SMMO_EINVAL for another work-group size or group. */
smmo_status smmo_set_launch(smmo_heap *h, uint32_t method_id, uint32_t class_id,
                            uint32_t wg_threads, uint32_t grid_waves, uint32_t group);

/* Method id of a method compiled into the library (names in smmo_methods.h),
 * SMMO_EINVAL if unknown. */
smmo_status smmo_method_id(const char *name, uint32_t *method_id);

/* Copies the last error message of the calling host thread (NUL-terminated,
 * truncated to n bytes). */
smmo_status smmo_last_error(char *buf, size_t n);

/* Hash of the sources the library was built from (every file of csrc/ and
 * include/, and the compiler flags), as a NUL-terminated hex string owned by
 * the library.  Bindings compare it with the sources beside them and refuse
 * a library built from other sources. */
const char *smmo_source_hash(void);

#ifdef __cplusplus
}
#endif
#endif /* SMMO_H */
