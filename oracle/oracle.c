/*
 * CPU oracle for the guest-memory translate-and-copy path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header or table with the GPU
 * library.
 *
 * What it computes (the software hybrid address space of section 4.2, "read
 * from / write to a user buffer at a guest virtual address"):
 *   - a guest virtual address is translated by walking the guest's own page
 *     tables in software to a guest-physical address (section 4.2), then the
 *     guest-physical address is turned into a host address through the VM's
 *     memslots, KVM's GPA-to-host map (section 4.2, citing KVM);
 *   - a buffer larger than a page is translated once per page, because pages
 *     contiguous in the guest need not be contiguous on the host (section 4.2);
 *   - a failing operation has altered nothing beyond what it already did and
 *     can be re-executed (section 6.6), so a copy stops at its first faulting
 *     page and reports how many bytes it moved.
 *
 * Page-table formats: x86-64 4-level and 5-level (48- and 57-bit linear
 * addresses), and the paper's own 32-bit PAE format (section 6.2; levels =
 * 3): CR3 bits 31:5 locate a 4-entry page-directory-pointer table indexed by
 * address bits 31:30, whose entries hold no permission or accessed bits;
 * below it the page directory and page table are the x86-64 ones.
 * Every point the paper leaves open follows the readings listed with the
 * design notes; the ones that shape this code are:
 *   - entry address bits are 51:12; XD, G, PWT, PCD, PAT and the available
 *     bits are ignored; bits 62:52 are ignored with 4/5 levels and reserved
 *     in PAE entries; CR3's low 12 bits are ignored (PAE: its low 5);
 *   - a PAE page-directory-pointer entry has bits 2:1, 8:5 and 63:52
 *     reserved, and is never given an accessed bit;
 *   - PS set in a level-4 or level-5 entry is reserved; a 2 MiB / 1 GiB leaf
 *     with any of bits [shift-1:13] set is reserved;
 *   - user-mode access: U/S must be 1 at every level, and R/W at every level
 *     for writes into the guest;
 *   - faults are reported top-down: table slot, present, reserved at each
 *     level; then user, write, and finally the data page's slot (level 0);
 *   - A (bit 5) is OR-ed into every entry of the walk of each page copied,
 *     and D (bit 6) into the leaf when the copy writes the guest; a walk that
 *     faults changes nothing;
 *   - the whole range must be user-canonical (below 2^47, 2^56 with 5
 *     levels, 2^32 with PAE) and must not wrap, else nothing happens; a
 *     zero-length copy does nothing and succeeds.
 *
 * Memory model: each VM owns one byte arena (host memory standing in for
 * the guest's RAM); a memslot maps [gpa, gpa+bytes) to [arena_off, ...).
 * Page tables live inside guest-physical memory and are read through the
 * memslots.  Request `host` fields are byte offsets into one host pool.
 * Everything is sequential and in request order.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum {
    ORC_OK = 0,
    ORC_NOT_PRESENT = 1,
    ORC_RESERVED = 2,
    ORC_PROT_USER = 3,
    ORC_PROT_WRITE = 4,
    ORC_NO_MEMSLOT = 5,
    ORC_NONCANONICAL = 6,
    ORC_INVALID = 7,
};

#define ORC_ADDR_MASK 0x000FFFFFFFFFF000ull
#define ORC_P 0x1ull
#define ORC_RW 0x2ull
#define ORC_US 0x4ull
#define ORC_A 0x20ull
#define ORC_D 0x40ull
#define ORC_PS 0x80ull

typedef struct { uint64_t gpa, bytes, arena_off; } orc_slot;

typedef struct {
    uint8_t *arena;
    uint64_t arena_bytes;
    const orc_slot *slots;
    uint32_t nslots;
} orc_vm;

typedef struct {
    uint32_t vm;
    uint32_t levels;
    uint64_t cr3;
} orc_proc;

typedef struct {
    orc_vm *vms;
    uint32_t nvm;
    orc_proc *procs;
    uint32_t nproc;
    uint8_t *pool;
    uint64_t pool_bytes;
    uint64_t n_ad_sets;      /* entries whose A or D bit this oracle turned on */
} orc_state;

/* 32-byte request, same field order as the library's descriptor. */
typedef struct {
    uint64_t gva;
    uint64_t host;           /* byte offset into the pool */
    uint32_t len;
    uint32_t asid;
    uint8_t dir;             /* 0: guest -> host, 1: host -> guest */
    uint8_t rsvd[3];
    uint32_t tag;
} orc_req;

typedef struct {
    uint64_t bytes_done;
    uint64_t fault_gva;
    uint32_t code;
    uint16_t level;
    uint16_t pad;
} orc_result;

typedef struct {
    uint64_t req_index;
    uint64_t fault_gva;
    uint32_t code;
    uint16_t level;
    uint16_t pad;
} orc_fault;

typedef struct {
    uint64_t gpa;
    uint64_t hpa;
    uint32_t code;
    uint8_t level;
    uint8_t page_shift;
    uint16_t vm;
} orc_xlat;

/* ---------------------------------------------------------------- state -- */
orc_state *orc_new(uint32_t nvm, uint32_t nproc) {
    orc_state *s = (orc_state *)calloc(1, sizeof(orc_state));
    if (!s) return NULL;
    s->vms = (orc_vm *)calloc(nvm ? nvm : 1, sizeof(orc_vm));
    s->procs = (orc_proc *)calloc(nproc ? nproc : 1, sizeof(orc_proc));
    s->nvm = nvm;
    s->nproc = nproc;
    return s;
}

void orc_free(orc_state *s) {
    if (!s) return;
    free(s->vms);
    free(s->procs);
    free(s);
}

void orc_set_vm(orc_state *s, uint32_t vm, uint8_t *arena, uint64_t arena_bytes,
                const orc_slot *slots, uint32_t nslots) {
    s->vms[vm].arena = arena;
    s->vms[vm].arena_bytes = arena_bytes;
    s->vms[vm].slots = slots;
    s->vms[vm].nslots = nslots;
}

void orc_set_proc(orc_state *s, uint32_t asid, uint32_t vm, uint64_t cr3, uint32_t levels) {
    s->procs[asid].vm = vm;
    s->procs[asid].cr3 = cr3;
    s->procs[asid].levels = levels;
}

void orc_set_pool(orc_state *s, uint8_t *pool, uint64_t bytes) {
    s->pool = pool;
    s->pool_bytes = bytes;
}

uint64_t orc_ad_sets(const orc_state *s) { return s->n_ad_sets; }

/* ------------------------------------------------------------- memslots -- */
/* GPA -> arena offset through the VM's memslots (section 4.2: KVM turns a
 * guest-physical address into the host address backing it).  Plain scan. */
static int slot_lookup(const orc_vm *v, uint64_t gpa, uint64_t *hpa) {
    for (uint32_t i = 0; i < v->nslots; i++) {
        const orc_slot *sl = &v->slots[i];
        if (gpa >= sl->gpa && gpa - sl->gpa < sl->bytes) {
            *hpa = sl->arena_off + (gpa - sl->gpa);
            return 1;
        }
    }
    return 0;
}

static uint64_t load64(const uint8_t *p) {
    uint64_t v = 0;
    for (int i = 7; i >= 0; i--) v = (v << 8) | p[i];   /* little endian */
    return v;
}

/* ----------------------------------------------------------------- walk -- */
typedef struct {
    uint32_t code;
    uint32_t level;         /* fault level, 0 when none or when the data page has no slot */
    uint32_t shift;         /* leaf page shift (12, 21, 30), 0 if no leaf was reached */
    uint32_t leaf_level;
    uint64_t gpa;           /* valid once a leaf was reached */
    uint64_t hpa;           /* arena offset, valid when code == OK */
    uint32_t npath;
    uint64_t path[5];       /* arena offsets of the entries read, top level first */
} walk_t;

/* Software walk of the guest page tables for one linear address
 * (section 4.2).  Precondition: the address is user-canonical. */
#define ORC_PAE_PDPTE_RSVD 0xFFF00000000001E6ull   /* bits 63:52, 8:5, 2:1 */
#define ORC_PAE_RSVD 0x7FF0000000000000ull         /* bits 62:52 of a PAE PDE/PTE */

static void walk(const orc_state *s, const orc_proc *p, uint64_t gva, int write, walk_t *w) {
    const orc_vm *v = &s->vms[p->vm];
    uint64_t table = p->cr3 & ORC_ADDR_MASK;
    int user_ok = 1, write_ok = 1;
    uint64_t frame = 0;
    int top = (int)p->levels;
    const int pae = p->levels == 3;
    memset(w, 0, sizeof(*w));
    if (pae) {
        /* the 4-entry table at CR3 bits 31:5; its entry is not part of the
         * accessed-bit path and grants every permission */
        uint64_t pdpt = p->cr3 & 0xFFFFFFE0ull;
        uint64_t thpa;
        if (!slot_lookup(v, pdpt, &thpa)) {
            w->code = ORC_NO_MEMSLOT;
            w->level = 3;
            return;
        }
        uint64_t e = load64(v->arena + thpa + 8 * ((gva >> 30) & 3));
        if (!(e & ORC_P)) {
            w->code = ORC_NOT_PRESENT;
            w->level = 3;
            return;
        }
        if (e & ORC_PAE_PDPTE_RSVD) {
            w->code = ORC_RESERVED;
            w->level = 3;
            return;
        }
        table = e & ORC_ADDR_MASK;
        top = 2;
    }
    for (int lvl = top; lvl >= 1; lvl--) {
        uint32_t shift = 12 + 9 * (uint32_t)(lvl - 1);
        uint64_t idx = (gva >> shift) & 511;
        uint64_t thpa;
        if (!slot_lookup(v, table, &thpa)) {
            w->code = ORC_NO_MEMSLOT;
            w->level = (uint32_t)lvl;
            return;
        }
        uint64_t eoff = thpa + 8 * idx;
        uint64_t e = load64(v->arena + eoff);
        w->path[w->npath++] = eoff;
        if (!(e & ORC_P)) {
            w->code = ORC_NOT_PRESENT;
            w->level = (uint32_t)lvl;
            return;
        }
        if (pae && (e & ORC_PAE_RSVD)) {
            w->code = ORC_RESERVED;
            w->level = (uint32_t)lvl;
            return;
        }
        user_ok &= (int)((e >> 2) & 1);
        write_ok &= (int)((e >> 1) & 1);
        if (lvl >= 4 && (e & ORC_PS)) {
            w->code = ORC_RESERVED;
            w->level = (uint32_t)lvl;
            return;
        }
        if ((lvl == 3 || lvl == 2) && (e & ORC_PS)) {
            uint64_t size = 1ull << shift;
            uint64_t rsvd = (size - 1) & ~((1ull << 13) - 1);   /* bits shift-1 .. 13 */
            if (e & rsvd) {
                w->code = ORC_RESERVED;
                w->level = (uint32_t)lvl;
                return;
            }
            frame = e & ORC_ADDR_MASK & ~(size - 1);
            w->shift = shift;
            w->leaf_level = (uint32_t)lvl;
            break;
        }
        if (lvl == 1) {
            frame = e & ORC_ADDR_MASK;
            w->shift = 12;
            w->leaf_level = 1;
            break;
        }
        table = e & ORC_ADDR_MASK;
    }
    w->gpa = frame | (gva & ((1ull << w->shift) - 1));
    if (!user_ok) {
        w->code = ORC_PROT_USER;
        w->level = w->leaf_level;
        return;
    }
    if (write && !write_ok) {
        w->code = ORC_PROT_WRITE;
        w->level = w->leaf_level;
        return;
    }
    if (!slot_lookup(v, w->gpa, &w->hpa)) {
        w->code = ORC_NO_MEMSLOT;
        w->level = 0;
        w->hpa = 0;
        return;
    }
    w->code = ORC_OK;
}

/* OR the accessed bit into every entry of the walk and, when writing, the
 * dirty bit into the leaf entry.  Bits only ever go from 0 to 1. */
static void set_ad(orc_state *s, const orc_proc *p, const walk_t *w, int write) {
    uint8_t *a = s->vms[p->vm].arena;
    for (uint32_t i = 0; i < w->npath; i++) {
        uint8_t want = (uint8_t)ORC_A;
        if (write && i + 1 == w->npath) want |= (uint8_t)ORC_D;
        if ((a[w->path[i]] & want) != want) s->n_ad_sets++;
        a[w->path[i]] |= want;
    }
}

static uint64_t user_limit(uint32_t levels) {
    return levels == 5 ? (1ull << 56) : levels == 3 ? (1ull << 32) : (1ull << 47);
}

/* ------------------------------------------------------------ translate -- */
#define ORC_XLAT_WRITE 1u
#define ORC_XLAT_SET_AD 2u

void orc_translate(orc_state *s, uint32_t asid, const uint64_t *gvas, uint64_t n, uint32_t flags,
                   orc_xlat *out) {
    for (uint64_t i = 0; i < n; i++) {
        orc_xlat *x = &out[i];
        memset(x, 0, sizeof(*x));
        if (asid >= s->nproc) {
            x->code = ORC_INVALID;
            x->vm = 0xFFFF;
            continue;
        }
        const orc_proc *p = &s->procs[asid];
        x->vm = (uint16_t)p->vm;
        if (gvas[i] >= user_limit(p->levels)) {
            x->code = ORC_NONCANONICAL;
            continue;
        }
        walk_t w;
        int write = (flags & ORC_XLAT_WRITE) != 0;
        walk(s, p, gvas[i], write, &w);
        x->code = w.code;
        x->level = (uint8_t)w.level;
        if (w.shift) {
            x->gpa = w.gpa;
            x->page_shift = (uint8_t)w.shift;
        }
        if (w.code == ORC_OK) {
            x->hpa = w.hpa;
            if (flags & ORC_XLAT_SET_AD) set_ad(s, p, &w, write);
        }
    }
}

/* ----------------------------------------------------------------- copy -- */
/* One copy between guest memory at req->gva and the pool at req->host,
 * page by page (section 4.2).  With move == 0 only the result is computed:
 * no byte moves and no A/D update (a result depends only on the page tables,
 * whose translation bits copies never change).  Returns -1 if the request
 * names pool bytes outside the pool (a caller error the tests never make). */
static int copy_req(orc_state *s, const orc_req *req, orc_result *res, int move) {
    memset(res, 0, sizeof(*res));
    if (req->asid >= s->nproc) {
        res->code = ORC_INVALID;
        res->fault_gva = req->gva;
        return 0;
    }
    if (req->len == 0) return 0;
    const orc_proc *p = &s->procs[req->asid];
    uint64_t lim = user_limit(p->levels);
    if (req->gva >= lim || (uint64_t)req->len > lim - req->gva) {
        res->code = ORC_NONCANONICAL;
        res->fault_gva = req->gva;
        return 0;
    }
    if (move && (req->host > s->pool_bytes || (uint64_t)req->len > s->pool_bytes - req->host)) return -1;
    int to_guest = req->dir != 0;
    uint8_t *arena = s->vms[p->vm].arena;
    uint64_t end = req->gva + req->len;
    for (uint64_t page = req->gva & ~0xFFFull; page < end; page += 4096) {
        uint64_t lo = page > req->gva ? page : req->gva;
        uint64_t hi = page + 4096 < end ? page + 4096 : end;
        walk_t w;
        walk(s, p, lo, to_guest, &w);
        if (w.code != ORC_OK) {
            res->bytes_done = lo - req->gva;
            res->fault_gva = lo;
            res->code = w.code;
            res->level = (uint16_t)w.level;
            return 0;
        }
        if (!move) continue;
        set_ad(s, p, &w, to_guest);
        uint8_t *g = arena + w.hpa;
        uint8_t *h = s->pool + req->host + (lo - req->gva);
        if (to_guest)
            memcpy(g, h, hi - lo);
        else
            memcpy(h, g, hi - lo);
    }
    res->bytes_done = req->len;
    return 0;
}

int orc_copy(orc_state *s, const orc_req *req, orc_result *res) { return copy_req(s, req, res, 1); }

/* A batch is its requests applied one after another in index order; the
 * fault list holds one record per request whose code is not OK, ascending
 * by request index.  Returns the number of faults, or -1 on a pool error. */
static int64_t batch(orc_state *s, const orc_req *reqs, uint64_t n, orc_result *res, orc_fault *faults, int move) {
    int64_t nf = 0;
    for (uint64_t i = 0; i < n; i++) {
        if (copy_req(s, &reqs[i], &res[i], move) != 0) return -1;
        if (res[i].code != ORC_OK) {
            if (faults) {
                faults[nf].req_index = i;
                faults[nf].fault_gva = res[i].fault_gva;
                faults[nf].code = res[i].code;
                faults[nf].level = res[i].level;
                faults[nf].pad = 0;
            }
            nf++;
        }
    }
    return nf;
}

int64_t orc_batch(orc_state *s, const orc_req *reqs, uint64_t n, orc_result *res, orc_fault *faults) {
    return batch(s, reqs, n, res, faults, 1);
}

/* Results and fault list of a batch, without moving bytes or touching A/D. */
int64_t orc_batch_results(orc_state *s, const orc_req *reqs, uint64_t n, orc_result *res, orc_fault *faults) {
    return batch(s, reqs, n, res, faults, 0);
}

/* ------------------------------------------------------ conflict checker -- */
/* The batch precondition: inside one epoch, no two requests touch
 * overlapping guest bytes (same VM) or overlapping pool bytes where at least
 * one of them writes, and no request copies into a page-table frame the
 * epoch walks.  This checker translates every page of every request with
 * the walk above (no side effects), collects byte intervals and sorts them.
 * Returns 0 when the batch is conflict-free, else 1 and the pair in *a, *b. */
typedef struct {
    uint64_t key;      /* vm (or 0xFFFFFFFF for the pool) */
    uint64_t lo, hi;
    uint64_t req;
    int write;
} ival;

static int ival_cmp(const void *x, const void *y) {
    const ival *a = (const ival *)x, *b = (const ival *)y;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->lo != b->lo) return a->lo < b->lo ? -1 : 1;
    return 0;
}

static int sweep(ival *v, uint64_t m, uint64_t *ra, uint64_t *rb) {
    qsort(v, m, sizeof(ival), ival_cmp);
    /* for each interval, compare with all earlier still-open intervals of the
     * same key; keep the furthest-reaching writer and reader seen so far */
    uint64_t cur_key = ~0ull;
    uint64_t w_hi = 0, w_req = 0, r_hi = 0, r_req = 0;
    for (uint64_t i = 0; i < m; i++) {
        if (v[i].key != cur_key) {
            cur_key = v[i].key;
            w_hi = r_hi = 0;
        }
        if (v[i].lo < w_hi && w_req != v[i].req) {
            *ra = w_req; *rb = v[i].req; return 1;
        }
        if (v[i].write && v[i].lo < r_hi && r_req != v[i].req) {
            *ra = r_req; *rb = v[i].req; return 1;
        }
        if (v[i].write) {
            if (v[i].hi > w_hi) { w_hi = v[i].hi; w_req = v[i].req; }
        } else {
            if (v[i].hi > r_hi) { r_hi = v[i].hi; r_req = v[i].req; }
        }
    }
    return 0;
}

int orc_check_conflicts(orc_state *s, const orc_req *reqs, uint64_t n, const uint64_t *epoch_end,
                        uint32_t n_epochs, uint64_t *ra, uint64_t *rb) {
    uint64_t start = 0;
    for (uint32_t e = 0; e < n_epochs || (n_epochs == 0 && start < n); e++) {
        uint64_t stop = n_epochs ? epoch_end[e] : n;
        /* per page: up to 5 walked entries + 1 data interval; per request: 1 pool interval */
        uint64_t cap = 1;
        for (uint64_t i = start; i < stop; i++) cap += 6 * (((uint64_t)reqs[i].len + 4095) / 4096 + 1) + 1;
        ival *v = (ival *)malloc(cap * sizeof(ival));
        if (!v) return -1;
        uint64_t m = 0;
        for (uint64_t i = start; i < stop; i++) {
            const orc_req *r = &reqs[i];
            if (r->asid >= s->nproc || r->len == 0) continue;
            const orc_proc *p = &s->procs[r->asid];
            uint64_t lim = user_limit(p->levels);
            if (r->gva >= lim || (uint64_t)r->len > lim - r->gva) continue;
            int to_guest = r->dir != 0;
            uint64_t end = r->gva + r->len, done = r->len;
            for (uint64_t page = r->gva & ~0xFFFull; page < end; page += 4096) {
                uint64_t lo = page > r->gva ? page : r->gva;
                uint64_t hi = page + 4096 < end ? page + 4096 : end;
                walk_t w;
                walk(s, p, lo, to_guest, &w);
                /* the walk's entries are read (and A/D OR-ed, which commutes) */
                for (uint32_t k = 0; k < w.npath; k++) {
                    v[m++] = (ival){p->vm, w.path[k], w.path[k] + 8, i, 0};
                }
                if (w.code != ORC_OK) { done = lo - r->gva; break; }
                v[m++] = (ival){p->vm, w.hpa, w.hpa + (hi - lo), i, to_guest};
            }
            if (done) v[m++] = (ival){0xFFFFFFFFull, r->host, r->host + done, i, !to_guest};
        }
        int bad = sweep(v, m, ra, rb);
        free(v);
        if (bad) return 1;
        start = stop;
        if (n_epochs == 0) break;
    }
    return 0;
}
