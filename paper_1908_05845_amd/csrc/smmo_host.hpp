// Host-side state of schemas and heaps, shared by the library's translation
// units.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/smmo.h"
#include "smmo_layout.hpp"

struct smmo_field_info {
    char name[32];
    int32_t dtype;
    uint32_t count;
    uint32_t size;       // bytes per element
    uint32_t offset;     // byte offset of element 0's 64-entry array in a block
    uint32_t stride;     // bytes from one inner element's array to the next
};

struct smmo_class_info {
    char name[32];
    uint32_t nfields;
    uint32_t narrays;
    smmo_field_info f[SMMO_MAX_FIELDS];
    uint32_t data_bytes;
    uint32_t parent = SMMO_NO_PARENT;
    uint32_t flags = 0;               // SMMO_CLASS_ABSTRACT
};

struct smmo_schema {
    uint32_t nclasses = 0;
    smmo_class_info c[SMMO_MAX_CLASSES];
    bool frozen = false;
};

namespace smmo {
// bit c set for every class c that is cls or derives from it
uint32_t class_family(const smmo_schema *s, uint32_t cls);
inline bool class_abstract(const smmo_schema *s, uint32_t cls) { return (s->c[cls].flags & SMMO_CLASS_ABSTRACT) != 0; }
} // namespace smmo

// Heaps of at most this many blocks walk the class of a stale list directly
// (every block, filtered by type) instead of enumerating it first, where
// methods create objects of the class (its list would be rebuilt launch
// after launch).
constexpr uint32_t kDirectMaxBlocks = 8192;

enum RState : int { R_DIRTY = 0, R_VALID = 1, R_SPLIT = 2 };   // R_SPLIT: valid, with the packing plan

// A method launch resolves its fields by name; the schema is frozen once a
// heap exists, so the resolved kernel parameters are cached per
// (method, class, argument bytes) to keep the host cost of a launch low.
struct smmo_bind_slot {
    const void *method = nullptr;
    uint32_t cls = 0;
    uint32_t nargs = 0;
    uint32_t nk = 0;
    alignas(8) unsigned char args[128];
    alignas(8) unsigned char k[256];
};

struct smmo_heap {
    smmo_schema *schema = nullptr;
    smmo::HeapView v{};
    void *base = nullptr;
    size_t bytes = 0;
    smmo_allocator owner{};            // set when base came from an allocator
    smmo_config cfg{};
    hipStream_t last = nullptr;
    int device = 0;
    uint64_t *host_ctrl = nullptr;     // pinned copy target for control words
    int rstate[SMMO_MAX_CLASSES] = {};
    // classes that methods create objects of (their lists go stale launch
    // after launch; small heaps walk them directly instead of re-enumerating)
    bool churn[SMMO_MAX_CLASSES] = {};
    // classes with a snapshot from smmo_snapshot that no do-all has used yet
    // (the list R of such a class is the snapshot's)
    uint32_t snap_pending = 0;
    uint64_t ub_blocks[SMMO_MAX_CLASSES] = {};   // upper bound of blocks per class
    uint32_t cu_count = 256;
    smmo_bind_slot bind_cache[16];
    uint32_t bind_next = 0;
    // launch shape per (method, class) set by smmo_set_launch (0 = default)
    uint16_t launch_wg[64][SMMO_MAX_CLASSES] = {};
    uint32_t launch_waves[64][SMMO_MAX_CLASSES] = {};
    uint8_t launch_group[64][SMMO_MAX_CLASSES] = {};
    uint32_t cur_method = 0xFFFFFFFFu;     // method being launched by smmo_parallel_do
    uint64_t defrag_nonce = 0;             // marks the source blocks of a defragmentation pass
};

namespace smmo {

// sets the calling thread's last-error text and returns `st`
smmo_status fail(smmo_status st, const std::string &msg);
smmo_status hip_fail(hipError_t e, const char *what);

uint32_t dtype_size(int32_t dtype);

// field lookup by name with the expected type and inner-array length
// (count 0 = any); on success fills offset / stride of the field
smmo_status bind_field(const smmo_schema *s, uint32_t cls, const char *name, int32_t dtype,
                       uint32_t count, uint32_t *offset, uint32_t *stride);

// block list of a class for the next launch: rebuilds it if it is stale;
// snapshot = copy allocation bitmaps to iteration bitmaps on the way; split =
// the list must carry the packing plan of packed do-alls: dense blocks at the
// front, sparse ones (at most 32 live objects) at the back (without it every
// block is listed as dense); allow_direct = a small heap's churning class may
// be walked over all blocks instead (false: the walk needs the list itself,
// its positions naming the class's blocks).
smmo_status ensure_enumerated(smmo_heap *h, uint32_t cls, bool snapshot, hipStream_t st, bool split = false,
                              bool allow_direct = true);


// launch shape of a do-all over class cls: the (method, class) setting of
// smmo_set_launch if any, else 256-thread work-groups and 64 wavefronts per
// CU, never more wavefronts than the class has groups of blocks; group =
// blocks a wavefront takes per iteration: 1 for a method without groups
// (def_group 0), else the setting, else the heap's block_group, else the
// method's default def_group
struct LaunchShape {
    dim3 grid;
    dim3 block;
    uint32_t group;
};
LaunchShape method_shape(const smmo_heap *h, uint32_t cls, uint32_t def_group = 0);

// whether a packed do-all of class cls launched with shape ls should get a
// list with the packing plan (sparse_packing 2, or 1 with a class that may
// have more blocks than the launch has wavefronts)
bool packing_wanted(const smmo_heap *h, uint32_t cls, const LaunchShape &ls);

// bookkeeping after a launch that creates objects of class cls (in_method:
// a method's device allocation, not a host-side bulk creation)
void note_allocation(smmo_heap *h, uint32_t cls, uint64_t max_new_objects, bool in_method = true);

struct MethodEntry {
    const char *name;
    size_t args_bytes;
    smmo_status (*launch)(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st);
    // kFamilyLaunch: a do-all on a class with descendants calls `launch` once
    // with the class itself, and the method covers the whole family in that
    // launch (it uses only fields every class of the family shares)
    uint32_t flags = 0;
};
constexpr uint32_t kFamilyLaunch = 1;

const MethodEntry *method_table(uint32_t *count);

// heap.hip helpers for the other translation units: class id check, control
// word read-back (synchronizes with the heap's last stream), launch error check
smmo_status heap_check_class(const smmo_heap *h, uint32_t cls);
smmo_status heap_read_ctrl(smmo_heap *h, uint32_t first_word, uint32_t nwords);
smmo_status heap_launch_check(const char *what);

} // namespace smmo
