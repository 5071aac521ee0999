/*
 * devirt.h -- C ABI of the MI355X (gfx950) guest-memory translate-and-copy
 * library.
 *
 * The library implements the data path of the software hybrid address space
 * (section 4.2 of "Making I/O Virtualization Easy with Device Files"): a host
 * driver that serves a guest's file operation reads or writes the guest's
 * user buffer at a guest virtual address.  Each page of the buffer is
 * translated separately, because guest-contiguous pages need not be
 * host-contiguous (section 4.2): first by a software walk of the guest's own
 * page tables (guest virtual -> guest physical), then through the VM's
 * memslots (guest physical -> host address, as KVM does; section 4.2).  The
 * bytes are then copied between the guest memory image and host buffers.
 *
 * Platform: x86-64 guest paging, 4-level (48-bit) or 5-level (57-bit), with
 * 4 KiB, 2 MiB and 1 GiB pages.  Guest memory ("arena") and host buffers
 * live in HBM of one GPU.  The paper's own platform was 32-bit PAE on KVM
 * (section 6.2); the interface below keeps its roles: a process is named by
 * its page-table root captured when it first issues an operation
 * (section 6.3), an operation carries a handful of scalar arguments
 * (section 6.1), results come back in a per-operation record (section 5), and
 * a failed operation leaves a defined, re-executable state (section 6.6).
 *
 * Conventions for every call:
 *   - Return value: 0 on success, a negative errno on misuse or a HIP failure
 *     (-EINVAL, -ENOMEM, -EEXIST, -EBUSY, -EIO, -ENOENT).  Calls never abort
 *     and never print; devirt_last_error() gives a message for the calling
 *     thread's last failure.
 *   - Guest faults are NOT errors: they are reported per operation in
 *     devirt_result / devirt_xlat / devirt_fault records.
 *   - Pointers named *_dev are device pointers (HBM of the context's GPU);
 *     *_host are host pointers.  The caller owns every buffer it passes and
 *     keeps it alive until the stream has passed the call.
 *   - Data-path calls (translate, copy, submit_batch) are asynchronous and
 *     ordered on the given HIP stream (NULL = the null stream).  Control
 *     calls (vm/memslot/process) synchronise the device first.
 *   - A context is externally synchronised: one thread at a time.
 */
#ifndef DEVIRT_H
#define DEVIRT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct devirt_ctx devirt_ctx;
typedef struct devirt_server devirt_server;

/* ---------------------------------------------------------------- records */

/* Direction of a copy (section 4.2: "read from and write to a user buffer"). */
#define DEVIRT_FROM_GUEST 0u /* guest memory -> host buffer (e.g. a guest write()) */
#define DEVIRT_TO_GUEST 1u   /* host buffer -> guest memory (e.g. a guest read())  */

/* One operation's argument buffer: 32 bytes, little endian, device memory.
 * Mirrors the few scalar arguments a forwarded file operation carries
 * (section 6.1). */
typedef struct {
    uint64_t gva;     /* guest virtual address of the buffer                */
    uint64_t host;    /* device pointer to the host-side buffer             */
    uint32_t len;     /* bytes                                              */
    uint32_t asid;    /* process id from devirt_process_create              */
    uint8_t dir;      /* DEVIRT_FROM_GUEST or DEVIRT_TO_GUEST               */
    uint8_t rsvd[3];  /* must be 0                                          */
    uint32_t tag;     /* caller's tag; the serving loop reads it as the
                         guest thread id (one operation in flight per id)  */
} devirt_request;

/* Fault codes (devirt_result.code, devirt_fault.code, devirt_xlat.code). */
#define DEVIRT_OK 0u
#define DEVIRT_NOT_PRESENT 1u  /* P = 0 in the entry at `level`                   */
#define DEVIRT_RESERVED 2u     /* PS in a level-4/5 entry, or a large leaf with
                                  bits [shift-1:13] set                           */
#define DEVIRT_PROT_USER 3u    /* U/S = 0 somewhere on the path (user access)     */
#define DEVIRT_PROT_WRITE 4u   /* R/W = 0 somewhere on the path, writing guest    */
#define DEVIRT_NO_MEMSLOT 5u   /* a table (level >= 1) or the data page (level 0)
                                  has no memslot                                  */
#define DEVIRT_NONCANONICAL 6u /* range not inside user canonical space, or wraps */
#define DEVIRT_INVALID 7u      /* unknown asid                                    */
#define DEVIRT_NO_POOL 8u      /* devirt_map_pages: too few pool frames for the
                                  tables the batch needs (nothing written)        */
#define DEVIRT_EPT_VIOLATION 9u /* VM with an EPT: a table (level >= 1) or the
                                  data page (level 0) is not present in the EPT,
                                  lacks a permission, or lies at or above 2^48    */
#define DEVIRT_EPT_MISCONFIG 10u /* VM with an EPT: a misconfigured EPT entry on
                                  the path (write without read, reserved bits,
                                  memory type 2/3/7) or one outside the arena     */

/* Per-operation result (24 bytes), the analogue of the per-guest-thread
 * result page (section 5).  Copies have prefix semantics: every byte before
 * the first faulting byte is copied, nothing after it; bytes_done is that
 * byte's offset.  fault_gva is the first byte not copied (0 if none). */
typedef struct {
    uint64_t bytes_done;
    uint64_t fault_gva;
    uint32_t code;
    uint16_t level;
    uint16_t pad;
} devirt_result;

/* Fault-list record (24 bytes): one per operation whose code is not OK,
 * ascending by request index. */
typedef struct {
    uint64_t req_index;
    uint64_t fault_gva;
    uint32_t code;
    uint16_t level;
    uint16_t pad;
} devirt_fault;

/* Translation of one address (24 bytes).  gpa and page_shift are set once a
 * leaf was reached (code OK, PROT_*, or NO_MEMSLOT at level 0); hpa (byte
 * offset in the VM's arena) only when code is OK; vm is 0xFFFF for an
 * unknown asid. */
typedef struct {
    uint64_t gpa;
    uint64_t hpa;
    uint32_t code;
    uint8_t level;
    uint8_t page_shift;
    uint16_t vm;
} devirt_xlat;

/* devirt_translate flags */
#define DEVIRT_XLAT_WRITE 1u  /* check write permission                          */
#define DEVIRT_XLAT_SET_AD 2u /* on success, OR A into every walked entry and,
                                 with WRITE, D into the leaf                     */

/* ---------------------------------------------------------------- context */

/* Open a context on HIP device `hip_device`.  A context plays the part of the
 * host-side backend of the common virtual driver (section 3.1): it holds the
 * guests' memory images, memslots and registered processes, and serves
 * forwarded operations against them.  -EIO if the device cannot be used. */
int devirt_open(int hip_device, devirt_ctx **out);
/* Release everything the context owns (arenas, tables, workspaces); waits
 * for the device first.  A server must have been stopped. */
int devirt_close(devirt_ctx *ctx);
/* Message for the calling thread's last failed call ("" if none). */
const char *devirt_last_error(void);

/* ------------------------------------------------- guest memory and tables */

/* Allocate a VM's guest-memory arena of `arena_bytes` (multiple of 4 KiB) in
 * HBM; returns its id in *vm.  The arena starts zeroed.  It stands for the
 * host memory that backs the guest's physical memory (section 2.2), which the
 * backend reads and writes at host addresses (section 4.2).  -ENOMEM if HBM
 * cannot hold it. */
int devirt_vm_create(devirt_ctx *ctx, uint64_t arena_bytes, uint32_t *vm);
/* Borrow the arena's device pointer and size (valid until devirt_close). */
int devirt_vm_arena(devirt_ctx *ctx, uint32_t vm, void **dev_ptr, uint64_t *bytes);
/* Synchronous copies into / out of an arena; src/dst may be host or device
 * pointers.  -EINVAL if [off, off+bytes) leaves the arena. */
int devirt_vm_write(devirt_ctx *ctx, uint32_t vm, uint64_t off, const void *src, uint64_t bytes);
int devirt_vm_read(devirt_ctx *ctx, uint32_t vm, uint64_t off, void *dst, uint64_t bytes);

/* Define memslot `slot` (0..63) of a VM: guest-physical [gpa, gpa+bytes) is
 * backed by arena bytes [arena_off, arena_off+bytes) (KVM's GPA -> host map,
 * section 4.2).  All three values 4 KiB aligned, gpa+bytes <= 2^52.
 * bytes == 0 deletes the slot.  -EEXIST if the GPA range overlaps another
 * slot of the VM, -EINVAL if unaligned or outside the arena. */
int devirt_memslot_set(devirt_ctx *ctx, uint32_t vm, uint32_t slot, uint64_t gpa, uint64_t bytes,
                       uint64_t arena_off);

/* Describe a VM's guest-physical space by a 4-level extended page table
 * instead of its memslots: the translation is then finished by a second
 * software walk, the paper's path for hypervisors other than KVM (section
 * 4.2; EPT in section 2.2).  root_arena_off: arena offset of the EPT's
 * level-4 table, 4 KiB aligned, inside the arena; ~0 returns the VM to its
 * memslots.  EPT tables live in the arena (the caller writes them with
 * devirt_vm_write); entry addresses are arena offsets.  Entry bits: 0 read,
 * 1 write, 2 execute (an entry with all three clear is not present), 5:3
 * memory type, 7 page size at levels 3 and 2 (1 GiB / 2 MiB leaves),
 * address 51:12; bits 63:52, 6, 8 and 9 are ignored and never written.
 * A guest page-table frame needs read and write through the EPT (the walk
 * may set A/D bits in it); a data page needs read when copied to the host or
 * translated for reading, write when copied into the guest or translated
 * with DEVIRT_XLAT_WRITE.  Failures report DEVIRT_EPT_VIOLATION or
 * DEVIRT_EPT_MISCONFIG at the guest level whose frame failed, 0 for the data
 * page.  -ENOENT for an unknown VM, -EINVAL for a bad root; waits for the
 * device to be idle, like devirt_memslot_set. */
int devirt_vm_set_ept(devirt_ctx *ctx, uint32_t vm, uint64_t root_arena_off);

/* Register a guest process by its page-table root (CR3) and paging mode,
 * captured once as the backend does when a thread first makes a call
 * (section 6.3).  levels 4 or 5: x86-64 4-level (48-bit) or 5-level (57-bit)
 * paging, CR3 low 12 bits ignored.  levels 3: 32-bit PAE paging, the paper's
 * own platform (section 6.2): CR3 bits 31:5 locate a 4-entry root table,
 * addresses stop at 2^32.  -EINVAL for any other depth.
 * Returns ids 0, 1, 2, ... */
int devirt_process_create(devirt_ctx *ctx, uint32_t vm, uint64_t cr3_gpa, uint32_t levels, uint32_t *asid);

/* ---------------------------------------------------------------- data path */

/* Translate n guest virtual addresses of process `asid` (section 4.2: walk
 * the guest page tables, then the memslots).  gva_dev: n x uint64_t;
 * out_dev: n x devirt_xlat. */
int devirt_translate(devirt_ctx *ctx, uint32_t asid, const uint64_t *gva_dev, uint64_t n, uint32_t flags,
                     devirt_xlat *out_dev, void *hip_stream);

/* One operation, one launch (the plain per-request method): copy len bytes
 * from guest memory at gva into dst_dev / from src_dev into guest memory at
 * gva, page by page (section 4.2), with prefix semantics on a fault and A/D
 * bits set for every page copied.  len < 2^32.  res_dev: 1 devirt_result. */
int devirt_copy_from_guest(devirt_ctx *ctx, uint32_t asid, uint64_t gva, void *dst_dev, uint64_t len,
                           devirt_result *res_dev, void *hip_stream);
int devirt_copy_to_guest(devirt_ctx *ctx, uint32_t asid, uint64_t gva, const void *src_dev, uint64_t len,
                         devirt_result *res_dev, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that must not call the allocator): the same copy as
 * devirt_copy_from_guest (dir = DEVIRT_FROM_GUEST, host_dev is the
 * destination) or devirt_copy_to_guest (dir = DEVIRT_TO_GUEST, host_dev is
 * the source), same results and effects, but its scratch (one request's queue
 * counters, clock origin and copy-segment queues) lives in a static device
 * array of about 1 MiB per device, looked up at devirt_open, and the call
 * allocates nothing.  The request may touch at most 16,384 4 KiB pages
 * (-EINVAL beyond, nothing done).  Every call on one device shares that
 * array: calls that overlap on one device (two streams, two contexts) race
 * and give undefined results; calls ordered on one stream do not.  Not
 * profiled (no timing events). */
int devirt_copy_static(devirt_ctx *ctx, uint32_t asid, uint64_t gva, void *host_dev, uint64_t len, uint32_t dir,
                       devirt_result *res_dev, void *hip_stream);

/* Map guest virtual pages by writing the guest's own page tables: the
 * second kind of routine of the software hybrid address space (section 4.2;
 * insert_pfn and kin), where the backend maps a page into the process
 * address space and takes the page-table pages it needs from guest-physical
 * frames the frontend handed over.
 *
 * maps_dev: n devirt_map (n <= 2^19).  Map i puts the 4 KiB page at gva
 * (aligned, in the user range) on the frame gpa (aligned, below 2^52): leaf
 * = gpa | P | U/S, plus R/W with DEVIRT_MAP_WRITE, A = D = 0.  When two maps
 * name one page, the later one wins.  Every walk sees the tables as they were
 * before the call.  Per map, res_dev (n devirt_result): OK with bytes_done =
 * 4096; NONCANONICAL (unaligned or out of range); RESERVED (a large leaf or
 * reserved bits on the path; `level` names it); NO_MEMSLOT (an existing table
 * outside every memslot); INVALID (unknown asid); NO_POOL.
 * New tables: each table the successful maps need and the process lacks is
 * created once, in order of level from the top down and ascending index
 * within a level, on pool_gpa_host[0], [1], ...: zeroed, then linked from its
 * parent entry with P, R/W and U/S (a PAE root entry: P only).  If n_pool is
 * too small, nothing is written and every map that would have succeeded
 * reports NO_POOL.  *n_used_dev (one uint64_t) receives the frames used.
 * pool_gpa_host: n_pool distinct, 4 KiB aligned frames inside memslots that
 * nothing else uses (-EINVAL otherwise); read before the call returns.
 * A VM with an EPT (devirt_vm_set_ept): the tables are read and written
 * through the EPT (a failure on the path reports DEVIRT_EPT_VIOLATION or
 * DEVIRT_EPT_MISCONFIG at its level), and pool frames need only be aligned
 * and distinct here: the frames the batch takes are translated through the
 * EPT on the device, and if one is not readable and writable there, nothing
 * is written and every map that would have succeeded reports NO_POOL.  The
 * EPT entries for the mapped frames themselves are the hypervisor's.
 * Asynchronous on hip_stream; no other call may touch the process's tables
 * meanwhile. */
typedef struct {
    uint64_t gva;
    uint64_t gpa;
    uint32_t flags; /* DEVIRT_MAP_WRITE */
    uint32_t pad;
} devirt_map;
#define DEVIRT_MAP_WRITE 1u
int devirt_map_pages(devirt_ctx *ctx, uint32_t asid, const devirt_map *maps_dev, uint64_t n,
                     const uint64_t *pool_gpa_host, uint64_t n_pool, devirt_result *res_dev, uint64_t *n_used_dev,
                     void *hip_stream);

/* The other half of mapping a page (section 4.2: the backend creates the
 * mapping in the guest page tables and also in the EPT, which the hypervisor
 * maintains): map guest-physical pages of VM `vm`, which must have an EPT
 * (devirt_vm_set_ept), by writing that EPT.
 *
 * maps_dev: n devirt_ept_map (n <= 2^19).  Map i puts the guest-physical
 * page at gpa (4 KiB-aligned, below 2^48) on the arena page at hpa (4 KiB-
 * aligned, inside the arena) with the rights in flags bits 2:0 (bit 0 read,
 * 1 write, 2 execute; not empty, no write without read, no other bit): a
 * 4 KiB EPT leaf = hpa | rights | memory type WB (6 << 3), replacing whatever
 * entry was there.  When two maps name one page, the later one wins.  Every
 * walk sees the EPT as it was before the call.  Per map, res_dev (n
 * devirt_result): OK with bytes_done = 4096; NONCANONICAL (bad gpa, hpa or
 * rights); RESERVED (a present 2 MiB / 1 GiB EPT leaf on the path: nothing is
 * split; `level` names it); EPT_MISCONFIG (a misconfigured EPT table entry on
 * the path, or a table outside the arena); NO_POOL.  fault_gva holds gpa for
 * a map that fails.
 * New EPT tables: each table the successful maps need and the EPT lacks is
 * created once, in order of level from the top down and ascending index
 * within a level, on pool_host[0], [1], ... (arena offsets): zeroed, then
 * linked from its parent entry with read, write and execute.  If n_pool is
 * too small, nothing is written and every map that would have succeeded
 * reports NO_POOL.  *n_used_dev (device) receives the pool pages used.
 * -EINVAL (nothing done): no such VM, a VM without an EPT, more than 2^19
 * maps, a pool page unaligned, outside the arena or repeated.  The pool pages
 * must not hold anything the guest or the EPT still uses (not checked).
 * Stream-ordered; the per-process translation caches are emptied. */
typedef struct {
    uint64_t gpa;
    uint64_t hpa;
    uint32_t flags; /* DEVIRT_EPT_R | DEVIRT_EPT_W | DEVIRT_EPT_X */
    uint32_t pad;
} devirt_ept_map;
#define DEVIRT_EPT_R 1u
#define DEVIRT_EPT_W 2u
#define DEVIRT_EPT_X 4u
int devirt_ept_map_pages(devirt_ctx *ctx, uint32_t vm, const devirt_ept_map *maps_dev, uint64_t n,
                         const uint64_t *pool_host, uint64_t n_pool, devirt_result *res_dev, uint64_t *n_used_dev,
                         void *hip_stream);

/* Many operations from many guests in one submission.  The paper forwards
 * one operation, a handful of scalar arguments, per hypercall (section 6.1),
 * and with dual threads the operations of different guest threads proceed
 * concurrently while each guest thread waits for its own (section 5); here
 * a whole batch of such operations is handed over at once.  Results equal
 * applying the requests one after another in index order, provided that
 * inside each epoch no two requests touch overlapping guest bytes of one VM
 * or overlapping host bytes where one of them writes, and that no request's
 * guest bytes, read or written, lie in a frame that any request of the batch
 * walks (a guest page table, a PAE root table or an EPT table); epochs run
 * in order (translation of an epoch may run ahead, during the copies of the
 * previous one, and ORs A/D bits meanwhile).  A violation gives undefined
 * bytes, never a fault of the library.  epoch_end_host: n_epochs ascending exclusive
 * end indices, the last == n (NULL: one epoch).  res_dev: n devirt_result;
 * faults_dev: room for n devirt_fault (may be NULL together with
 * n_faults_dev); n_faults_dev: one uint64_t; t_done_dev: NULL or n uint64_t
 * receiving each request's completion time in ns after the submission
 * started on the device. */
int devirt_submit_batch(devirt_ctx *ctx, const devirt_request *reqs_dev, uint64_t n,
                        const uint64_t *epoch_end_host, uint32_t n_epochs, devirt_result *res_dev,
                        devirt_fault *faults_dev, uint64_t *n_faults_dev, uint64_t *t_done_dev, void *hip_stream);

/* Wait for everything the context enqueued on hip_stream: the blocking use of
 * the data path, where the caller sleeps until its operations are done
 * (section 5).  -EIO on a HIP failure. */
int devirt_sync(devirt_ctx *ctx, void *hip_stream);

/* ---------------------------------------------------------------- tuning */

/* Launch and schedule knobs of the batched path.  None changes results. */
typedef struct {
    uint32_t group;           /* requests one translating wavefront owns: 1..64     */
    uint32_t seg_chunks;      /* max 4 KiB pages merged into one copy segment: 1..64 */
    uint32_t xlat_wg;         /* translate workgroup size (multiple of 64, <= 256)  */
    uint32_t xlat_wgs_per_cu; /* translate grid = CUs x this                        */
    uint32_t copy_wg;         /* copy workgroup size (multiple of 64, <= 1024)      */
    uint32_t copy_wgs_per_cu; /* copy grid = CUs x this                             */
    uint32_t nontemporal;     /* 1: streaming (non-temporal) stores when copying     */
    uint32_t inline_bytes;    /* segments up to this size (<= 256) are copied by the
                                 translating lane itself                            */
    uint32_t use_graph;       /* 1: capture each distinct batch shape as a HIP graph
                                 and replay it                                     */
    uint32_t overlap;         /* 1: translate epoch e+1 on a second stream while
                                 epoch e is being copied                          */
    uint32_t fifo_entries;    /* per-request path: entries of each process's FIFO
                                 translation cache (section 4.2 uses 10), 0..16;
                                 0 = no cache (see devirt_fifo_counts)             */
    uint32_t large_pages;     /* batched path: a request of more pages than this is
                                 walked by the 4 wavefronts of a workgroup
                                 together; 0 (the default) = every request by
                                 one wavefront; else >= 64                         */
    uint32_t spill_side;      /* with overlap: 1 (the default) = the spill pass of
                                 epoch e (groups whose runs overflowed the queue)
                                 and the fault list run on the translate stream,
                                 beside copy(e) and ahead of translate(e+1); 0 =
                                 on the copy stream, right after copy(e) and at
                                 the end                                          */
} devirt_config;

int devirt_get_config(devirt_ctx *ctx, devirt_config *cfg);
/* -EINVAL if a field is out of range; the previous config is kept. */
int devirt_set_config(devirt_ctx *ctx, const devirt_config *cfg);

/* Time candidate configs on a real batch and keep the fastest.  The batch
 * is executed once per candidate and repetition, with the usual effects on
 * guest memory, host buffers, A/D bits and result buffers; the final state
 * is that of the last execution.  The winner is stored in the context and
 * returned in *best (and its median time in *best_ms).  Synchronous. */
int devirt_autotune(devirt_ctx *ctx, const devirt_request *reqs_dev, uint64_t n, const uint64_t *epoch_end_host,
                    uint32_t n_epochs, devirt_result *res_dev, devirt_fault *faults_dev, uint64_t *n_faults_dev,
                    void *hip_stream, uint32_t reps, devirt_config *best, double *best_ms);

/* devirt_autotune with a persistent cache of its winners.  cache_path_host:
 * a text file, one JSON object per line, {"key": ..., "ms": ..., "config":
 * {...}}; the key is the device (architecture name and CU count) and
 * workload_key_host (the caller's name for the batch's shape, without quotes,
 * backslashes or newlines).  If the file holds the key (the last such line
 * wins), its config is set and returned with its recorded time, nothing is
 * executed and *hit = 1.  Otherwise devirt_autotune runs (same effects) and a
 * line is appended; *hit = 0.  -EIO if the file cannot be written. */
int devirt_autotune_cached(devirt_ctx *ctx, const char *cache_path_host, const char *workload_key_host,
                           const devirt_request *reqs_dev, uint64_t n, const uint64_t *epoch_end_host,
                           uint32_t n_epochs, devirt_result *res_dev, devirt_fault *faults_dev,
                           uint64_t *n_faults_dev, void *hip_stream, uint32_t reps, devirt_config *best,
                           double *best_ms, int *hit);

/* The per-process translation cache of section 4.2 (the backend keeps each
 * guest process's recent translations in a FIFO of 10 entries).  With
 * devirt_config.fifo_entries = k > 0, the per-request calls (devirt_copy_*)
 * look each page they translate up in the process's k-entry FIFO, in page
 * order, up to and including the first faulting page.  A lookup hits when the
 * 4 KiB page is held and, for a copy into the guest, was filled or last
 * refreshed by such a copy; a hit skips the page walk (its A/D bits are
 * already set).  A miss walks; a successful walk inserts the page at the
 * tail, evicting the oldest entry when full (or marks a held entry written);
 * hits never reorder; failed walks insert nothing.  Results are the same with
 * and without the cache.  Any devirt_vm_write, memslot, EPT, process or
 * devirt_map_pages call empties every cache (counts are kept); a caller that
 * writes page tables through the devirt_vm_arena pointer must call
 * devirt_fifo_flush.  Per-request calls of one process must be ordered (one
 * stream) while the cache is on.  The batched and serving paths do not use
 * it.
 * devirt_fifo_counts: the process's hits and misses since the last flush
 * (synchronises the device); -ENOENT for an unknown asid.
 * devirt_fifo_flush: empty every process's cache and zero its counts. */
int devirt_fifo_counts(devirt_ctx *ctx, uint32_t asid, uint64_t *hits, uint64_t *misses);
int devirt_fifo_flush(devirt_ctx *ctx);

/* ---------------------------------------------------------------- metrics */

typedef struct {
    uint64_t batches;        /* devirt_submit_batch calls                          */
    uint64_t epochs;         /* epochs launched                                    */
    uint64_t plain_calls;    /* devirt_copy_* calls                                */
    uint64_t graph_replays;  /* batches served by replaying a captured graph       */
    /* the following are filled only while profiling (timing, then counters) */
    uint64_t copy_launches;  /* copy-kernel launches timed                         */
    double copy_ms;          /* summed copy-kernel time (HIP events)               */
    uint64_t xlat_launches;  /* translate-kernel launches timed                    */
    double xlat_ms;          /* summed translate-kernel time                       */
    uint64_t pages_walked;   /* 4 KiB pages translated by the batched path         */
    uint64_t cache_hits;     /* per-wavefront walk-cache hits (1 GiB regions)      */
    uint64_t cache_misses;
    uint64_t segments;       /* copy segments queued                               */
    uint64_t inline_segments;/* segments copied by the translating wavefront       */
    uint64_t ad_atomics;     /* A/D atomic ORs issued                              */
    uint64_t spilled_groups; /* request groups whose runs overflowed the segment
                                queue while an earlier epoch was being copied:
                                translated again and copied after that epoch's
                                copy (the spill pass)                              */
    uint64_t large_requests; /* requests walked by a workgroup (large_pages)      */
} devirt_stats;

/* Profiling flags.  While any is set, data-path calls run without graphs.
 *  DEVIRT_PROF_TIMING:   each kernel launch is bracketed by HIP events on the
 *                        call's stream (copy_ms, xlat_ms and launch counts);
 *  DEVIRT_PROF_COUNTERS: the kernels also gather device counters (pages,
 *                        cache hits, segments, A/D ORs).  Gathering them costs
 *                        atomics on shared addresses, so kernel times taken
 *                        with this flag are pessimistic.
 * devirt_get_stats synchronises to read them.  -EINVAL for unknown flags. */
#define DEVIRT_PROF_TIMING 1
#define DEVIRT_PROF_COUNTERS 2
int devirt_set_profiling(devirt_ctx *ctx, int flags);
int devirt_get_stats(devirt_ctx *ctx, devirt_stats *out);
int devirt_reset_stats(devirt_ctx *ctx);

/* ---------------------------------------------------------------- serving */

/* Serving loop: operations arrive one by one and are admitted when (a) their
 * guest thread (devirt_request.tag, per asid) has no operation in flight --
 * the guest thread sleeps until its operation completes (section 5) -- (b) a
 * descriptor slot is free and (c) the bytes of all operations in flight stay
 * within pool_bytes.  Admitted operations are batched continuously: while
 * earlier batches run on the GPU, newly admitted ones are launched on further
 * streams.  Page tables stay resident in the context.
 *
 * How the server learns that a batch has finished (flags):
 *  DEVIRT_SERVE_POLL     the server thread polls each batch's event (section
 *                        7.4 finds polling faster than interrupts);
 *  DEVIRT_SERVE_NOTIFY   a host function enqueued after each batch marks it
 *                        done and wakes the server thread, which sleeps while
 *                        batches run (the interrupt-style completion);
 *  DEVIRT_SERVE_BLOCKING the server waits for each batch before it admits
 *                        anything else: one batch at a time, no overlap (the
 *                        blocking mode of section 5).
 * Results do not depend on the mode.  DEVIRT_SERVE_DEVICE_TIMES may be OR-ed
 * into the mode: each batch is then bracketed by timing events on its
 * stream, and every completion carries its batch's window on the device
 * clock (dev_start_ns, dev_end_ns); two batches whose windows overlap were
 * executing on the GPU at the same time. */
#define DEVIRT_SERVE_POLL 0u
#define DEVIRT_SERVE_NOTIFY 1u
#define DEVIRT_SERVE_BLOCKING 2u
#define DEVIRT_SERVE_DEVICE_TIMES 0x100u
typedef struct {
    uint32_t max_inflight; /* descriptor slots (operations admitted, not yet done)  */
    uint64_t pool_bytes;   /* byte budget of operations in flight                   */
    uint32_t max_batch;    /* operations per launch (0: max_inflight)               */
    uint32_t streams;      /* launches in flight at once, 1..8                      */
    uint32_t flags;        /* completion mode: one DEVIRT_SERVE_* mode, optionally
                              | DEVIRT_SERVE_DEVICE_TIMES                          */
} devirt_server_cfg;

typedef struct {
    uint64_t ticket;       /* submission order, from 0                              */
    devirt_result res;
    uint64_t t_submit_ns;  /* host steady clock: submitted                          */
    uint64_t t_admit_ns;   /* admitted into a launch                                */
    uint64_t t_done_ns;    /* completion observed by the server                     */
    uint64_t dev_start_ns; /* DEVIRT_SERVE_DEVICE_TIMES: the batch's window on the
                              device, ns after the server started (else 0)        */
    uint64_t dev_end_ns;
} devirt_completion;

/* Start a server thread on the context.  While it runs, the context may
 * only be used through the server (and read-only queries). */
int devirt_server_start(devirt_ctx *ctx, const devirt_server_cfg *cfg, devirt_server **out);
/* Queue n operations (host copies of the descriptors; their host buffers are
 * device memory the caller keeps alive until completion).  Returns the
 * number queued in *n_queued; -EBUSY if the queue is full. */
int devirt_server_submit(devirt_server *srv, const devirt_request *reqs_host, uint32_t n, uint32_t *n_queued);
/* Queue a map batch as an operation of guest thread (asid, tag): the
 * backend mapping pages into the process between the thread's forwarded
 * copies (section 4.2; the batch is what devirt_map_pages does, with the same
 * map records, pool rules and per-map results).  It runs in the thread's
 * order, after every earlier operation of the thread has completed, and
 * alone: once every batch already on the GPU has finished, with nothing
 * admitted until it is done, since a table write must not race a walk.
 * maps_host (n records, 8-byte aligned) and pool_gpa_host are copied at the
 * call; res_host (n records, 8-byte aligned) receives every map's result when
 * the batch completes and must stay alive until then.  Its completion
 * summarizes the batch: bytes_done = 4096 per map that succeeded; code, level
 * and fault_gva of the first map that failed (DEVIRT_OK if none).  *ticket
 * (may be NULL) receives its ticket.  A bad pool (unaligned, repeated, outside
 * every memslot) or more than 2^19 maps is refused here with -EINVAL. */
int devirt_server_submit_map(devirt_server *srv, uint32_t asid, uint32_t tag, const devirt_map *maps_host,
                             uint32_t n, const uint64_t *pool_gpa_host, uint32_t n_pool,
                             devirt_result *res_host, uint64_t *ticket);
/* The same for an EPT map batch of VM vm (devirt_ept_map_pages: the mapping
 * the hypervisor creates in the EPT, section 4.2), ordered as an operation of
 * guest thread (asid, tag) and run alone in the same way.  The summary's
 * fault_gva is the first failed map's guest-physical page.  An unknown VM, a
 * VM without an EPT or a bad pool (unaligned, outside the arena, repeated) is
 * refused here with -EINVAL. */
int devirt_server_submit_ept_map(devirt_server *srv, uint32_t asid, uint32_t tag, uint32_t vm,
                                 const devirt_ept_map *maps_host, uint32_t n, const uint64_t *pool_host,
                                 uint32_t n_pool, devirt_result *res_host, uint64_t *ticket);
/* Take up to max completions (any order); *n_out receives the count. */
int devirt_server_poll(devirt_server *srv, devirt_completion *out, uint32_t max, uint32_t *n_out);
/* Drain: wait until everything submitted has completed. */
int devirt_server_drain(devirt_server *srv);
/* Stop the thread (after draining) and free the server. */
int devirt_server_stop(devirt_server *srv);

/* Where the server thread's time goes (cumulative since start; host clock). */
typedef struct {
    uint64_t loops;        /* iterations of the server loop                         */
    uint64_t launches;     /* batches launched                                      */
    uint64_t ops;          /* operations completed                                  */
    uint64_t ns_inbox;     /* moving submitted operations into guest-thread FIFOs   */
    uint64_t ns_complete;  /* polling slot events and turning results into
                              completions                                          */
    uint64_t ns_admit;     /* admission and writing descriptors                     */
    uint64_t ns_launch;    /* enqueueing the kernels of a batch                     */
    uint64_t direct_launches; /* small batches run as one kernel that translates and
                                 copies (at most 64 operations, 256 KiB, 64 KiB each) */
} devirt_server_stats;
/* Read the counters (any thread; values may be a few iterations old). */
int devirt_server_get_stats(devirt_server *srv, devirt_server_stats *out);

#ifdef __cplusplus
}
#endif
#endif /* DEVIRT_H */
