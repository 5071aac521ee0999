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
 * Everything is sequential and in request order, except orc_batch_mt: it
 * splits each epoch's requests over threads, which the batch precondition
 * (no two requests of an epoch touch overlapping bytes where one writes, no
 * request touches a walked table frame) makes equivalent.  For that case
 * entry bytes are loaded and A/D bits OR-ed with relaxed byte atomics; the
 * bits a walk decides on never change during a batch.
 *
 * A VM may instead have its guest-physical space described by a 4-level
 * extended page table (EPT) kept in its arena: the translation is then
 * finished by a second software walk, as the paper prescribes for
 * hypervisors other than KVM (section 4.2; EPT itself in section 2.2).  The
 * readings that shape that walk:
 *   - EPT entries: bits 2:0 read, write, execute; not present when all three
 *     are 0; address bits 51:12; bit 7 makes a level-3 / level-2 entry a
 *     1 GiB / 2 MiB leaf; bits 63:52, the ignore-PAT bit and the accessed /
 *     dirty bits are ignored, and this walker sets no EPT bit;
 *   - misconfigured (EPT_MISCONFIG): write without read; any of bits 7:3 in
 *     a table entry; a leaf memory type (bits 5:3) of 2, 3 or 7; a large
 *     leaf with any of bits [shift-1:12] set; a table or page that does not
 *     lie inside the arena;
 *   - EPT_VIOLATION: a not-present entry, a guest-physical address at or
 *     above 2^48, or a missing permission: the read and write bits are
 *     AND-ed over the walk; a guest page-table frame needs both (the walk
 *     may write A/D bits into it, and hardware with EPT A/D enabled treats
 *     such accesses as writes), a data page needs read when copied to the
 *     host and write when copied into the guest;
 *   - per level, top-down: present, then misconfiguration; permissions once
 *     the leaf is reached; the reported level is the guest level whose
 *     frame failed (0 for the data page), as for a missing memslot;
 *   - mapping pages in such a VM reads and writes the guest's tables through
 *     the EPT, and translates the pool frames the batch takes through it
 *     too: if one of them is not readable and writable, nothing is written
 *     and every map that would have succeeded reports NO_POOL.
 */
#include <pthread.h>
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
    ORC_NO_POOL = 8,
    ORC_EPT_VIOLATION = 9,
    ORC_EPT_MISCONFIG = 10,
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
    int has_ept;             /* translate through the EPT at ept_root instead of the memslots */
    uint64_t ept_root;       /* arena offset of the EPT's level-4 table */
} orc_vm;

typedef struct {
    uint32_t vm;
    uint32_t levels;
    uint64_t cr3;
} orc_proc;

/* A process's translation cache (see "translation cache" below). */
#define ORC_FIFO_MAX 64
typedef struct {
    uint64_t vpn[ORC_FIFO_MAX];   /* slot i holds virtual page vpn[i]           */
    uint8_t writable[ORC_FIFO_MAX];
    uint32_t n;                   /* entries held                               */
    uint32_t head;                /* slot of the oldest entry                   */
    uint64_t hits, misses;
} orc_fifo;

typedef struct {
    orc_vm *vms;
    uint32_t nvm;
    orc_proc *procs;
    uint32_t nproc;
    uint8_t *pool;
    uint64_t pool_bytes;
    uint64_t n_ad_sets;      /* entries whose A or D bit this oracle turned on */
    orc_fifo *fifo;          /* per process; NULL while the cache is off        */
    uint32_t fifo_entries;
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
    free(s->fifo);
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

/* Give a VM an EPT rooted at arena offset `root` (4 KiB aligned, inside the
 * arena), or take it away with root = ~0.  Returns -1 on a bad root. */
int orc_set_ept(orc_state *s, uint32_t vm, uint64_t root) {
    orc_vm *v = &s->vms[vm];
    if (root == ~0ull) {
        v->has_ept = 0;
        return 0;
    }
    if ((root & 0xFFF) || root >= v->arena_bytes || v->arena_bytes - root < 4096) return -1;
    v->has_ept = 1;
    v->ept_root = root;
    return 0;
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
    for (int i = 7; i >= 0; i--) v = (v << 8) | __atomic_load_n(&p[i], __ATOMIC_RELAXED);   /* little endian */
    return v;
}

/* ------------------------------------------------------------------ EPT -- */
#define ORC_NEED_R 1u
#define ORC_NEED_W 2u
#define ORC_NEED_TABLE (ORC_NEED_R | ORC_NEED_W)

/* 1 if the 4 KiB page at arena offset `off` lies inside the arena. */
static int in_arena(const orc_vm *v, uint64_t off) {
    return off < v->arena_bytes && v->arena_bytes - off >= 4096;
}

/* Arena offsets of every table entry a walk loads (guest tables at every
 * level, the PAE root table, EPT tables).  Only the conflict checker asks
 * for them; every other caller passes NULL. */
typedef struct {
    uint32_t n;
    uint64_t off[40];
} reads_t;

static void note_read(reads_t *rec, uint64_t off) {
    if (rec && rec->n < 40) rec->off[rec->n++] = off;
}

/* GPA -> arena offset by walking the VM's EPT (see the header comment). */
static uint32_t ept_walk(const orc_vm *v, uint64_t gpa, uint32_t need, uint64_t *hpa, reads_t *rec) {
    if (gpa >> 48) return ORC_EPT_VIOLATION;
    uint64_t table = v->ept_root;
    int can_r = 1, can_w = 1;
    for (int lvl = 4; lvl >= 1; lvl--) {
        uint32_t eshift = 12u + 9u * (uint32_t)(lvl - 1);
        uint64_t eoff = table + 8 * ((gpa >> eshift) & 511);
        note_read(rec, eoff);
        uint64_t e = load64(v->arena + eoff);
        if ((e & 7) == 0) return ORC_EPT_VIOLATION;
        if ((e & 3) == 2) return ORC_EPT_MISCONFIG;
        can_r &= (int)(e & 1);
        can_w &= (int)((e >> 1) & 1);
        int leaf = lvl == 1 || ((lvl == 3 || lvl == 2) && (e & 0x80));
        if (!leaf) {
            if (e & 0xF8) return ORC_EPT_MISCONFIG;
            table = e & ORC_ADDR_MASK;
            if (!in_arena(v, table)) return ORC_EPT_MISCONFIG;
            continue;
        }
        uint64_t mt = (e >> 3) & 7;
        if (mt == 2 || mt == 3 || mt == 7) return ORC_EPT_MISCONFIG;
        uint64_t size = 1ull << eshift;
        if (e & (size - 1) & ~0xFFFull) return ORC_EPT_MISCONFIG;
        uint64_t h = (e & ORC_ADDR_MASK) | (gpa & (size - 1));
        if (!in_arena(v, h & ~0xFFFull)) return ORC_EPT_MISCONFIG;
        if (((need & ORC_NEED_R) && !can_r) || ((need & ORC_NEED_W) && !can_w)) return ORC_EPT_VIOLATION;
        *hpa = h;
        return ORC_OK;
    }
    return ORC_EPT_VIOLATION;   /* not reached */
}

/* GPA -> arena offset for an access that needs `need`: the EPT walk, or the
 * memslots when the VM has no EPT. */
static uint32_t gpa_to_hpa_rec(const orc_vm *v, uint64_t gpa, uint32_t need, uint64_t *hpa, reads_t *rec) {
    if (v->has_ept) return ept_walk(v, gpa, need, hpa, rec);
    return slot_lookup(v, gpa, hpa) ? ORC_OK : ORC_NO_MEMSLOT;
}

static uint32_t gpa_to_hpa(const orc_vm *v, uint64_t gpa, uint32_t need, uint64_t *hpa) {
    return gpa_to_hpa_rec(v, gpa, need, hpa, NULL);
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

static void walk_rec(const orc_state *s, const orc_proc *p, uint64_t gva, int write, walk_t *w, reads_t *rec) {
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
        uint32_t c = gpa_to_hpa_rec(v, pdpt, ORC_NEED_TABLE, &thpa, rec);
        if (c != ORC_OK) {
            w->code = c;
            w->level = 3;
            return;
        }
        uint64_t roff = thpa + 8 * ((gva >> 30) & 3);
        note_read(rec, roff);
        uint64_t e = load64(v->arena + roff);
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
        uint32_t c = gpa_to_hpa_rec(v, table, ORC_NEED_TABLE, &thpa, rec);
        if (c != ORC_OK) {
            w->code = c;
            w->level = (uint32_t)lvl;
            return;
        }
        uint64_t eoff = thpa + 8 * idx;
        note_read(rec, eoff);
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
    uint32_t c = gpa_to_hpa_rec(v, w->gpa, write ? ORC_NEED_W : ORC_NEED_R, &w->hpa, rec);
    if (c != ORC_OK) {
        w->code = c;
        w->level = 0;
        w->hpa = 0;
        return;
    }
    w->code = ORC_OK;
}

static void walk(const orc_state *s, const orc_proc *p, uint64_t gva, int write, walk_t *w) {
    walk_rec(s, p, gva, write, w, NULL);
}

/* OR the accessed bit into every entry of the walk and, when writing, the
 * dirty bit into the leaf entry.  Bits only ever go from 0 to 1. */
static void set_ad(orc_state *s, const orc_proc *p, const walk_t *w, int write) {
    uint8_t *a = s->vms[p->vm].arena;
    for (uint32_t i = 0; i < w->npath; i++) {
        uint8_t want = (uint8_t)ORC_A;
        if (write && i + 1 == w->npath) want |= (uint8_t)ORC_D;
        uint8_t old = __atomic_fetch_or(&a[w->path[i]], want, __ATOMIC_RELAXED);
        if ((old & want) != want) __atomic_fetch_add(&s->n_ad_sets, 1, __ATOMIC_RELAXED);
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

/* ---------------------------------------------------- translation cache -- */
/* Section 4.2: the backend caches the translations it makes, per guest
 * process, in a FIFO of 10 entries, the way a TLB caches page-table walks.
 * The cache changes no result (a hit gives the translation a walk would give:
 * the tables change only in A/D bits during a run); what it adds is the count
 * of translations served from it.  Readings:
 *   - an entry is one 4 KiB virtual page of the process, and records whether
 *     the walk that filled or last refreshed it was a write;
 *   - every page a copy translates (in order, up to and including its first
 *     faulting page) is one lookup; it hits when the page is held and, for a
 *     write into the guest, its entry records a write;
 *   - a miss walks; if the walk succeeds the page is inserted at the tail,
 *     evicting the oldest entry when the FIFO is full, or, if the page is
 *     already held (a write after reads), its entry is marked written in
 *     place; a hit changes nothing (FIFO, not LRU); a failed walk inserts
 *     nothing.
 * orc_fifo_reset turns the cache on with `entries` slots per process (0: off)
 * and empties it, as a change to the tables must. */
int orc_fifo_reset(orc_state *s, uint32_t entries) {
    if (entries > ORC_FIFO_MAX) return -1;
    free(s->fifo);
    s->fifo = NULL;
    s->fifo_entries = entries;
    if (entries) {
        s->fifo = (orc_fifo *)calloc(s->nproc ? s->nproc : 1, sizeof(orc_fifo));
        if (!s->fifo) return -1;
    }
    return 0;
}

void orc_fifo_counts(const orc_state *s, uint32_t asid, uint64_t *hits, uint64_t *misses) {
    *hits = *misses = 0;
    if (!s->fifo || asid >= s->nproc) return;
    *hits = s->fifo[asid].hits;
    *misses = s->fifo[asid].misses;
}

/* Slot holding `vpn`, or -1. */
static int fifo_find(const orc_fifo *f, uint32_t entries, uint64_t vpn) {
    for (uint32_t k = 0; k < f->n; k++) {
        uint32_t slot = (f->head + k) % entries;
        if (f->vpn[slot] == vpn) return (int)slot;
    }
    return -1;
}

/* One lookup; ok: the page's walk succeeded.  Returns 1 on a hit. */
static int fifo_lookup(orc_state *s, uint32_t asid, uint64_t vpn, int write, int ok) {
    orc_fifo *f = &s->fifo[asid];
    const uint32_t cap = s->fifo_entries;
    int slot = fifo_find(f, cap, vpn);
    if (slot >= 0 && (!write || f->writable[slot])) {
        f->hits++;
        return 1;
    }
    f->misses++;
    if (!ok) return 0;
    if (slot >= 0) {
        f->writable[slot] = 1;
        return 0;
    }
    uint32_t tail = (f->head + f->n) % cap;
    if (f->n == cap) {
        tail = f->head;  /* the oldest entry leaves */
        f->head = (f->head + 1) % cap;
    } else {
        f->n++;
    }
    f->vpn[tail] = vpn;
    f->writable[tail] = (uint8_t)(write != 0);
    return 0;
}

/* ----------------------------------------------------------------- copy -- */
/* What a copy does besides computing its result. */
enum {
    ORC_MOVE_NONE = 0,  /* result only: no byte moves, no A/D update          */
    ORC_MOVE_ALL = 1,   /* A/D update and byte moves: the operation itself    */
    ORC_MOVE_AD = 2,    /* A/D update only (the page-table side of the copy)  */
};

/* One copy between guest memory at req->gva and the pool at req->host,
 * page by page (section 4.2).  A result depends only on the page tables,
 * whose translation bits copies never change, so the three modes above give
 * the same result.  Returns -1 if the request names pool bytes outside the
 * pool (a caller error the tests never make). */
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
    if (move == ORC_MOVE_ALL && (req->host > s->pool_bytes || (uint64_t)req->len > s->pool_bytes - req->host))
        return -1;
    int to_guest = req->dir != 0;
    uint8_t *arena = s->vms[p->vm].arena;
    uint64_t end = req->gva + req->len;
    for (uint64_t page = req->gva & ~0xFFFull; page < end; page += 4096) {
        uint64_t lo = page > req->gva ? page : req->gva;
        uint64_t hi = page + 4096 < end ? page + 4096 : end;
        walk_t w;
        walk(s, p, lo, to_guest, &w);
        if (s->fifo) fifo_lookup(s, req->asid, lo >> 12, to_guest, w.code == ORC_OK);
        if (w.code != ORC_OK) {
            res->bytes_done = lo - req->gva;
            res->fault_gva = lo;
            res->code = w.code;
            res->level = (uint16_t)w.level;
            return 0;
        }
        if (move == ORC_MOVE_NONE) continue;
        set_ad(s, p, &w, to_guest);
        if (move == ORC_MOVE_AD) continue;
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

int orc_copy(orc_state *s, const orc_req *req, orc_result *res) { return copy_req(s, req, res, ORC_MOVE_ALL); }

/* The fault list: one record per request whose code is not OK, ascending by
 * request index.  Returns the number of faults. */
static int64_t fault_list(const orc_result *res, uint64_t n, orc_fault *faults) {
    int64_t nf = 0;
    for (uint64_t i = 0; i < n; i++) {
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

/* A batch is its requests applied one after another in index order.
 * Returns the number of faults, or -1 on a pool error. */
static int64_t batch(orc_state *s, const orc_req *reqs, uint64_t n, orc_result *res, orc_fault *faults, int move) {
    for (uint64_t i = 0; i < n; i++)
        if (copy_req(s, &reqs[i], &res[i], move) != 0) return -1;
    return fault_list(res, n, faults);
}

int64_t orc_batch(orc_state *s, const orc_req *reqs, uint64_t n, orc_result *res, orc_fault *faults) {
    return batch(s, reqs, n, res, faults, ORC_MOVE_ALL);
}

/* Results and fault list of a batch, without moving bytes or touching A/D. */
int64_t orc_batch_results(orc_state *s, const orc_req *reqs, uint64_t n, orc_result *res, orc_fault *faults) {
    return batch(s, reqs, n, res, faults, ORC_MOVE_NONE);
}

/* Results, fault list and the A/D bits of a batch, without moving payload
 * bytes: the final page-table frames equal those after orc_batch. */
int64_t orc_batch_ad(orc_state *s, const orc_req *reqs, uint64_t n, orc_result *res, orc_fault *faults) {
    return batch(s, reqs, n, res, faults, ORC_MOVE_AD);
}

/* The same batch on several threads: epochs in order, the requests of one
 * epoch split into `nthreads` contiguous slices, one thread each.  Under the
 * batch precondition the final state equals orc_batch's (move = 1) or
 * orc_batch_ad's (move = 2).  epoch_end: n_epochs ascending exclusive ends,
 * the last == n.  Returns the number of faults, -1 on a pool error, -3 if
 * the epoch ends do not finish at n, -4 while the translation cache is on.
 * A slice no thread can be started for runs on the calling thread. */
typedef struct {
    orc_state *s;
    const orc_req *reqs;
    orc_result *res;
    uint64_t lo, hi;
    int move, rc;
} slice_t;

static void *run_slice(void *arg) {
    slice_t *t = (slice_t *)arg;
    for (uint64_t i = t->lo; i < t->hi && t->rc == 0; i++)
        if (copy_req(t->s, &t->reqs[i], &t->res[i], t->move) != 0) t->rc = -1;
    return NULL;
}

int64_t orc_batch_mt(orc_state *s, const orc_req *reqs, uint64_t n, const uint64_t *epoch_end, uint32_t n_epochs,
                     uint32_t nthreads, int move, orc_result *res, orc_fault *faults) {
    if (s->fifo) return -4;  /* the translation cache is defined in request order only */
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    slice_t t[256];
    pthread_t th[256];
    int started[256];
    uint64_t r0 = 0;
    for (uint32_t e = 0; e < n_epochs; e++) {
        const uint64_t r1 = epoch_end[e];
        const uint64_t m = r1 - r0;
        for (uint32_t j = 0; j < nthreads; j++) {
            t[j].s = s;
            t[j].reqs = reqs;
            t[j].res = res;
            t[j].lo = r0 + m * j / nthreads;
            t[j].hi = r0 + m * (j + 1) / nthreads;
            t[j].move = move;
            t[j].rc = 0;
            started[j] = j + 1 < nthreads && t[j].hi > t[j].lo &&
                         pthread_create(&th[j], NULL, run_slice, &t[j]) == 0;
        }
        for (uint32_t j = 0; j < nthreads; j++)  /* the last slice, and any no thread took */
            if (!started[j]) run_slice(&t[j]);
        int rc = 0;
        for (uint32_t j = 0; j < nthreads; j++) {
            if (started[j]) pthread_join(th[j], NULL);
            if (t[j].rc) rc = t[j].rc;
        }
        if (rc) return rc;
        r0 = r1;
    }
    if (r0 != n) return -3;
    return fault_list(res, n, faults);
}

/* ------------------------------------------------------ conflict checker -- */
/* The batch precondition, in two rules.
 *   1. Inside one epoch, no two requests touch overlapping guest bytes (same
 *      VM) or overlapping pool bytes where at least one of them writes.
 *   2. Across the whole batch, no request's guest bytes (read or written)
 *      lie in a frame that holds an entry some walk of the batch loads: a
 *      guest page table at any level, the PAE root table, an EPT table.
 * Rule 2 spans epochs because a batched run may translate one epoch while
 * the previous one is being copied, and it covers reads too because walks
 * OR accessed/dirty bits into the entries they load.  For rule 2 every page
 * of a request's range is walked, including pages after its first fault,
 * since a parallel run translates a request's pages side by side.
 * The checker walks with the walker above (no side effects), collects byte
 * intervals and table frames and sorts them.  Returns 0 when the batch
 * meets both rules, 1 with the offending pair in *ra, *rb (for rule 2: the
 * request whose bytes lie in the table, then a request whose walk loads
 * it), -1 when out of memory. */
typedef struct {
    uint64_t key;      /* vm (or 0xFFFFFFFF for the pool) */
    uint64_t lo, hi;
    uint64_t req;
    int write;
} ival;

typedef struct {
    uint64_t vm, frame, req;
} tframe;

static int ival_cmp(const void *x, const void *y) {
    const ival *a = (const ival *)x, *b = (const ival *)y;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->lo != b->lo) return a->lo < b->lo ? -1 : 1;
    return 0;
}

static int tframe_cmp(const void *x, const void *y) {
    const tframe *a = (const tframe *)x, *b = (const tframe *)y;
    if (a->vm != b->vm) return a->vm < b->vm ? -1 : 1;
    if (a->frame != b->frame) return a->frame < b->frame ? -1 : 1;
    return 0;
}

/* Rule 1 for one epoch's intervals. */
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
        /* an earlier writer: a conflict with any request, itself included (one
         * request's intervals share its direction, so two of them overlapping
         * under a writer are two writes of aliased guest pages) */
        if (v[i].lo < w_hi) {
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

/* Sort and deduplicate the table frames collected so far (one walker kept per frame). */
static uint64_t compact_frames(tframe *t, uint64_t m) {
    if (m == 0) return 0;
    qsort(t, m, sizeof(tframe), tframe_cmp);
    uint64_t k = 1;
    for (uint64_t i = 1; i < m; i++)
        if (t[i].vm != t[k - 1].vm || t[i].frame != t[k - 1].frame) t[k++] = t[i];
    return k;
}

int orc_check_conflicts(orc_state *s, const orc_req *reqs, uint64_t n, const uint64_t *epoch_end,
                        uint32_t n_epochs, uint64_t *ra, uint64_t *rb) {
    int rc = 0;
    /* rule 2 material, whole batch: table frames walked, guest byte intervals */
    uint64_t tcap = 1024, nt = 0, gcap = 1024, ng = 0;
    tframe *tf = (tframe *)malloc(tcap * sizeof(tframe));
    ival *gi = (ival *)malloc(gcap * sizeof(ival));
    ival *v = NULL;
    if (!tf || !gi) { rc = -1; goto out; }
    uint64_t start = 0;
    for (uint32_t e = 0; e < n_epochs || (n_epochs == 0 && start < n); e++) {
        uint64_t stop = n_epochs ? epoch_end[e] : n;
        /* rule 1: per page 1 data interval; per request 1 pool interval */
        uint64_t cap = 1;
        for (uint64_t i = start; i < stop; i++) cap += ((uint64_t)reqs[i].len + 4095) / 4096 + 2;
        v = (ival *)malloc(cap * sizeof(ival));
        if (!v) { rc = -1; goto out; }
        uint64_t m = 0;
        for (uint64_t i = start; i < stop; i++) {
            const orc_req *r = &reqs[i];
            if (r->asid >= s->nproc || r->len == 0) continue;
            const orc_proc *p = &s->procs[r->asid];
            uint64_t lim = user_limit(p->levels);
            if (r->gva >= lim || (uint64_t)r->len > lim - r->gva) continue;
            int to_guest = r->dir != 0;
            uint64_t end = r->gva + r->len, done = r->len;
            int faulted = 0;
            for (uint64_t page = r->gva & ~0xFFFull; page < end; page += 4096) {
                uint64_t lo = page > r->gva ? page : r->gva;
                uint64_t hi = page + 4096 < end ? page + 4096 : end;
                walk_t w;
                reads_t rd;
                rd.n = 0;
                walk_rec(s, p, lo, to_guest, &w, &rd);
                for (uint32_t k = 0; k < rd.n; k++) {
                    if (nt == tcap) {
                        nt = compact_frames(tf, nt);
                        if (nt * 2 > tcap) {
                            tframe *g = (tframe *)realloc(tf, 2 * tcap * sizeof(tframe));
                            if (!g) { rc = -1; goto out; }
                            tf = g;
                            tcap *= 2;
                        }
                    }
                    tf[nt++] = (tframe){p->vm, rd.off[k] & ~0xFFFull, i};
                }
                if (faulted) continue;
                if (w.code != ORC_OK) { faulted = 1; done = lo - r->gva; continue; }
                ival d = {p->vm, w.hpa, w.hpa + (hi - lo), i, to_guest};
                v[m++] = d;
                if (ng == gcap) {
                    ival *g = (ival *)realloc(gi, 2 * gcap * sizeof(ival));
                    if (!g) { rc = -1; goto out; }
                    gi = g;
                    gcap *= 2;
                }
                gi[ng++] = d;
            }
            if (done) v[m++] = (ival){0xFFFFFFFFull, r->host, r->host + done, i, !to_guest};
        }
        int bad = sweep(v, m, ra, rb);
        free(v);
        v = NULL;
        if (bad) { rc = 1; goto out; }
        start = stop;
        if (n_epochs == 0) break;
    }
    /* rule 2: does any guest byte interval touch a walked table frame? */
    nt = compact_frames(tf, nt);
    for (uint64_t i = 0; i < ng; i++) {
        /* the first frame of this VM at or above the interval's first frame */
        uint64_t lo = 0, hi = nt, f0 = gi[i].lo & ~0xFFFull;
        while (lo < hi) {
            uint64_t mid = (lo + hi) / 2;
            if (tf[mid].vm < gi[i].key || (tf[mid].vm == gi[i].key && tf[mid].frame < f0))
                lo = mid + 1;
            else
                hi = mid;
        }
        if (lo < nt && tf[lo].vm == gi[i].key && tf[lo].frame < gi[i].hi) {
            *ra = gi[i].req;
            *rb = tf[lo].req;
            rc = 1;
            goto out;
        }
    }
out:
    free(v);
    free(tf);
    free(gi);
    return rc;
}

/* ------------------------------------------------------------ map pages -- */
/* The second kind of routine of the software hybrid address space (section
 * 4.2): map a page into the process address space by writing the guest's own
 * page tables, taking new table pages from guest-physical frames the
 * frontend handed over.  Batched, with this definition:
 *   - map i puts the 4 KiB page at gva (aligned, user range) on the frame at
 *     gpa (aligned, below 2^52): leaf = gpa | P | U/S, plus R/W when
 *     flags & 1; when two maps name one page, the later one wins;
 *   - every walk runs on the tables as they were before the call.  A present
 *     large leaf or reserved bits on the path fail the map (RESERVED), so does
 *     an existing table outside every memslot (NO_MEMSLOT);
 *   - the tables the successful maps lack are created once each, in order of
 *     level from the top down and ascending index within a level, on the pool
 *     frames in order; each is zeroed and linked from its parent entry with P,
 *     R/W and U/S (a PAE root entry: P only);
 *   - if the pool is too small nothing is written and every map that would
 *     have succeeded reports NO_POOL.
 * Returns the number of pool frames used; -1 if a pool frame is unaligned or
 * outside every memslot. */
typedef struct {
    uint64_t gva, gpa;
    uint32_t flags, pad;
} orc_map;

static int cmp_u64(const void *a, const void *b) {
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : x > y;
}

static uint64_t map_key(uint32_t level, uint64_t gva) {
    return ((uint64_t)(8 - level) << 56) | (gva >> (12 + 9 * level));
}

/* Walk for a map (no A/D).  On success *missing is the highest level whose
 * entry is not present (the tables below it are lacking), 0 if none is. */
static uint32_t map_walk(const orc_state *s, const orc_proc *p, uint64_t gva, uint32_t *level,
                         uint32_t *missing) {
    const orc_vm *v = &s->vms[p->vm];
    const int pae = p->levels == 3;
    uint64_t table = pae ? (p->cr3 & 0xFFFFFFE0ull) : (p->cr3 & ORC_ADDR_MASK);
    *missing = 0;
    for (int lvl = (int)p->levels; lvl >= 2; lvl--) {
        uint64_t thpa;
        uint32_t c = gpa_to_hpa(v, table, ORC_NEED_TABLE, &thpa);
        if (c != ORC_OK) {
            *level = (uint32_t)lvl;
            return c;
        }
        uint64_t idx = (pae && lvl == 3) ? ((gva >> 30) & 3) : ((gva >> (12 + 9 * (lvl - 1))) & 511);
        uint64_t e = load64(v->arena + thpa + 8 * idx);
        if (!(e & ORC_P)) {
            *missing = (uint32_t)lvl;
            return ORC_OK;
        }
        int rsvd = pae ? (lvl == 3 ? (e & ORC_PAE_PDPTE_RSVD) != 0 : (e & ORC_PAE_RSVD) != 0) : 0;
        if (rsvd || (!(pae && lvl == 3) && (e & ORC_PS))) {  /* reserved, or a large leaf on the path */
            *level = (uint32_t)lvl;
            return ORC_RESERVED;
        }
        table = e & ORC_ADDR_MASK;
    }
    uint64_t thpa;
    uint32_t c = gpa_to_hpa(v, table, ORC_NEED_TABLE, &thpa);   /* the page table itself */
    if (c != ORC_OK) {
        *level = 1;
        return c;
    }
    return ORC_OK;
}

/* Arena offset of the existing table at `level` on gva's path (the walk to it
 * is known to succeed), or of the PAE root table when level is the top. */
static uint64_t existing_table(const orc_state *s, const orc_proc *p, uint64_t gva, uint32_t level) {
    const orc_vm *v = &s->vms[p->vm];
    const int pae = p->levels == 3;
    uint64_t table = pae ? (p->cr3 & 0xFFFFFFE0ull) : (p->cr3 & ORC_ADDR_MASK);
    uint64_t hpa = 0;
    for (int lvl = (int)p->levels; lvl > (int)level; lvl--) {
        gpa_to_hpa(v, table, ORC_NEED_TABLE, &hpa);
        uint64_t idx = (pae && lvl == 3) ? ((gva >> 30) & 3) : ((gva >> (12 + 9 * (lvl - 1))) & 511);
        table = load64(v->arena + hpa + 8 * idx) & ORC_ADDR_MASK;
    }
    gpa_to_hpa(v, table, ORC_NEED_TABLE, &hpa);
    return hpa;
}

static void store64(uint8_t *p, uint64_t v) {
    for (int i = 0; i < 8; i++) p[i] = (uint8_t)(v >> (8 * i));
}

int64_t orc_map_pages(orc_state *s, uint32_t asid, const orc_map *maps, uint64_t n, const uint64_t *pool,
                      uint64_t n_pool, orc_result *res) {
    if (asid >= s->nproc) {
        for (uint64_t i = 0; i < n; i++) {
            memset(&res[i], 0, sizeof(res[i]));
            res[i].code = ORC_INVALID;
            res[i].fault_gva = maps[i].gva;
        }
        return 0;
    }
    const orc_proc *p = &s->procs[asid];
    orc_vm *v = &s->vms[p->vm];
    const int pae = p->levels == 3;
    uint64_t *pool_hpa = (uint64_t *)malloc((n_pool ? n_pool : 1) * sizeof(uint64_t));
    /* memslot VM: every frame must lie in a memslot (an error otherwise);
     * EPT VM: frames are translated below, once the batch's needs are known */
    for (uint64_t k = 0; k < n_pool; k++)
        if ((pool[k] & 0xFFF) || (!v->has_ept && !slot_lookup(v, pool[k], &pool_hpa[k]))) {
            free(pool_hpa);
            return -1;
        }
    /* 1. walk every map on the initial tables; gather the lacking tables */
    uint64_t *keys = (uint64_t *)malloc((4 * n + 1) * sizeof(uint64_t));
    uint64_t nk = 0;
    const uint64_t lim = user_limit(p->levels);
    for (uint64_t i = 0; i < n; i++) {
        const orc_map *m = &maps[i];
        orc_result *r = &res[i];
        memset(r, 0, sizeof(*r));
        if ((m->gva & 0xFFF) || m->gva >= lim || (m->gpa & 0xFFF) || m->gpa >= (1ull << 52)) {
            r->code = ORC_NONCANONICAL;
            r->fault_gva = m->gva;
            continue;
        }
        uint32_t level = 0, missing = 0;
        uint32_t code = map_walk(s, p, m->gva, &level, &missing);
        if (code != ORC_OK) {
            r->code = code;
            r->level = (uint16_t)level;
            r->fault_gva = m->gva;
            continue;
        }
        r->bytes_done = 4096;
        for (uint32_t l = missing ? missing - 1 : 0; l >= 1; l--) keys[nk++] = map_key(l, m->gva);
    }
    qsort(keys, nk, sizeof(uint64_t), cmp_u64);
    uint64_t nt = 0;
    for (uint64_t k = 0; k < nk; k++)
        if (nt == 0 || keys[nt - 1] != keys[k]) keys[nt++] = keys[k];
    int short_pool = nt > n_pool;
    /* EPT VM: the frames the batch takes must be readable and writable
     * through the EPT, like every table frame; else it is as if the pool
     * were short */
    for (uint64_t k = 0; v->has_ept && !short_pool && k < nt; k++)
        if (gpa_to_hpa(v, pool[k], ORC_NEED_TABLE, &pool_hpa[k]) != ORC_OK) short_pool = 1;
    if (short_pool) {   /* 2. not enough usable frames: nothing is written */
        for (uint64_t i = 0; i < n; i++)
            if (res[i].code == ORC_OK) {
                res[i].code = ORC_NO_POOL;
                res[i].bytes_done = 0;
                res[i].fault_gva = maps[i].gva;
            }
        free(keys);
        free(pool_hpa);
        return 0;
    }
    /* 3. new tables: zeroed, then linked from their parents */
    for (uint64_t k = 0; k < nt; k++) memset(v->arena + pool_hpa[k], 0, 4096);
    for (uint64_t k = 0; k < nt; k++) {
        uint32_t l = 8 - (uint32_t)(keys[k] >> 56);
        uint64_t id = keys[k] & ((1ull << 56) - 1);
        uint64_t va = id << (12 + 9 * l);
        uint64_t parent_key = map_key(l + 1, va), phpa;
        /* the parent is new unless it is the root table */
        uint64_t *hit = l + 1 < (uint32_t)p->levels
                            ? (uint64_t *)bsearch(&parent_key, keys, nt, sizeof(uint64_t), cmp_u64)
                            : NULL;
        if (hit)
            phpa = pool_hpa[hit - keys];
        else
            phpa = existing_table(s, p, va, l + 1);
        int root_pae = pae && l + 1 == 3;
        uint64_t idx = root_pae ? ((va >> 30) & 3) : (id & 511);
        uint64_t e = pool[k] | (root_pae ? ORC_P : (ORC_P | ORC_RW | ORC_US));
        store64(v->arena + phpa + 8 * idx, e);
    }
    /* 4. leaves, in index order */
    for (uint64_t i = 0; i < n; i++) {
        if (res[i].code != ORC_OK) continue;
        const orc_map *m = &maps[i];
        uint64_t key = map_key(1, m->gva), pt;
        uint64_t *hit = nt ? (uint64_t *)bsearch(&key, keys, nt, sizeof(uint64_t), cmp_u64) : NULL;
        pt = hit ? pool_hpa[hit - keys] : existing_table(s, p, m->gva, 1);
        uint64_t e = m->gpa | ORC_P | ORC_US | ((m->flags & 1) ? ORC_RW : 0);
        store64(v->arena + pt + 8 * ((m->gva >> 12) & 511), e);
    }
    free(keys);
    free(pool_hpa);
    return (int64_t)nt;
}

/* ------------------------------------------------------- EPT map pages -- */
/* The other half of the second kind of routine (section 4.2): the backend
 * creates the mapping in the guest page tables and also in the EPT, which
 * the hypervisor maintains.  Here the EPT half, batched, for a VM whose
 * guest-physical space is described by an EPT:
 *   - map i puts the guest-physical page at gpa (aligned, below 2^48) on the
 *     arena page at hpa (aligned, inside the arena), with the permissions in
 *     flags bits 2:0 (R, W, X; not empty, no write without read): leaf =
 *     hpa | perms | WB memory type (6 << 3); a 4 KiB leaf, replacing whatever
 *     entry was there; when two maps name one page, the later one wins;
 *   - anything else (other flag bits included) is NONCANONICAL;
 *   - every walk runs on the tables as they were before the call.  A present
 *     1 GiB or 2 MiB leaf on the path fails the map (RESERVED at its level:
 *     nothing is split); a misconfigured table entry on the path (write
 *     without read, bits 7:3 set, a table outside the arena) fails it with
 *     EPT_MISCONFIG at that level;
 *   - the tables the successful maps lack are created once each, in order of
 *     level from the top down and ascending index within a level, on the pool
 *     pages (arena offsets) in order; each is zeroed and linked from its
 *     parent entry with R, W and X;
 *   - if the pool is too small nothing is written and every map that would
 *     have succeeded reports NO_POOL.
 * Returns the number of pool pages used; -1 if the VM has no EPT or a pool
 * page is unaligned, outside the arena or repeated. */
typedef struct {
    uint64_t gpa, hpa;
    uint32_t flags, pad;
} orc_ept_map;

#define ORC_EPT_RWX 7ull
#define ORC_EPT_WB (6ull << 3)

static uint64_t ept_entry_off(uint64_t table, uint32_t level, uint64_t gpa) {
    return table + 8 * ((gpa >> (12 + 9 * (level - 1))) & 511);
}

/* Walk for an EPT map.  On success *missing is the highest level whose entry
 * is not present (the tables below it are lacking), 0 if the page table
 * exists. */
static uint32_t ept_map_walk(const orc_vm *v, uint64_t gpa, uint32_t *level, uint32_t *missing) {
    uint64_t table = v->ept_root;
    *missing = 0;
    for (uint32_t lvl = 4; lvl >= 2; lvl--) {
        uint64_t e = load64(v->arena + ept_entry_off(table, lvl, gpa));
        if ((e & 7) == 0) {
            *missing = lvl;
            return ORC_OK;
        }
        *level = lvl;
        if ((e & 3u) == 2u) return ORC_EPT_MISCONFIG;          /* write without read */
        if (lvl <= 3 && (e & 0x80)) return ORC_RESERVED;      /* a large leaf on the path */
        if (e & 0xF8u) return ORC_EPT_MISCONFIG;               /* bits 7:3 of a table entry */
        table = e & ORC_ADDR_MASK;
        if (!in_arena(v, table)) return ORC_EPT_MISCONFIG;     /* a table outside the arena */
    }
    *level = 0;
    return ORC_OK;
}

/* Arena offset of the existing EPT table at `level` on gpa's path (the path
 * to it is known to be present). */
static uint64_t existing_ept_table(const orc_vm *v, uint64_t gpa, uint32_t level) {
    uint64_t table = v->ept_root;
    for (uint32_t lvl = 4; lvl > level; lvl--) table = load64(v->arena + ept_entry_off(table, lvl, gpa)) & ORC_ADDR_MASK;
    return table;
}

int64_t orc_ept_map_pages(orc_state *s, uint32_t vm, const orc_ept_map *maps, uint64_t n, const uint64_t *pool,
                          uint64_t n_pool, orc_result *res) {
    if (vm >= s->nvm || !s->vms[vm].has_ept) return -1;
    orc_vm *v = &s->vms[vm];
    for (uint64_t k = 0; k < n_pool; k++) {
        if ((pool[k] & 0xFFF) || !in_arena(v, pool[k])) return -1;
        for (uint64_t j = 0; j < k; j++)
            if (pool[j] == pool[k]) return -1;
    }
    /* 1. walk every map on the initial EPT; gather the lacking tables */
    uint64_t *keys = (uint64_t *)malloc((3 * n + 1) * sizeof(uint64_t));
    uint64_t nk = 0;
    for (uint64_t i = 0; i < n; i++) {
        const orc_ept_map *m = &maps[i];
        orc_result *r = &res[i];
        memset(r, 0, sizeof(*r));
        const uint32_t perms = m->flags & 7u;
        if ((m->gpa & 0xFFF) || (m->gpa >> 48) || (m->hpa & 0xFFF) || !in_arena(v, m->hpa) || (m->flags & ~7u) ||
            perms == 0 || (perms & 3u) == 2u) {
            r->code = ORC_NONCANONICAL;
            r->fault_gva = m->gpa;
            continue;
        }
        uint32_t level = 0, missing = 0;
        uint32_t code = ept_map_walk(v, m->gpa, &level, &missing);
        if (code != ORC_OK) {
            r->code = code;
            r->level = (uint16_t)level;
            r->fault_gva = m->gpa;
            continue;
        }
        r->bytes_done = 4096;
        for (uint32_t l = missing ? missing - 1 : 0; l >= 1; l--) keys[nk++] = map_key(l, m->gpa);
    }
    qsort(keys, nk, sizeof(uint64_t), cmp_u64);
    uint64_t nt = 0;
    for (uint64_t k = 0; k < nk; k++)
        if (nt == 0 || keys[nt - 1] != keys[k]) keys[nt++] = keys[k];
    if (nt > n_pool) {   /* 2. not enough pool pages: nothing is written */
        for (uint64_t i = 0; i < n; i++)
            if (res[i].code == ORC_OK) {
                res[i].code = (uint32_t)ORC_NO_POOL;   /* would have succeeded */
                res[i].bytes_done = 0;
                res[i].fault_gva = maps[i].gpa;
            }
        free(keys);
        return 0;
    }
    /* 3. new tables: zeroed, then linked from their parents */
    for (uint64_t k = 0; k < nt; k++) memset(v->arena + pool[k], 0, 4096);
    for (uint64_t k = 0; k < nt; k++) {
        uint32_t l = 8 - (uint32_t)(keys[k] >> 56);
        uint64_t id = keys[k] & ((1ull << 56) - 1);
        uint64_t gpa = id << (12 + 9 * l);
        uint64_t parent_key = map_key(l + 1, gpa), parent;
        /* the parent is new unless it is the level-4 table */
        uint64_t *hit = l + 1 < 4 ? (uint64_t *)bsearch(&parent_key, keys, nt, sizeof(uint64_t), cmp_u64) : NULL;
        parent = hit ? pool[hit - keys] : existing_ept_table(v, gpa, l + 1);
        store64(v->arena + ept_entry_off(parent, l + 1, gpa), pool[k] | ORC_EPT_RWX);
    }
    /* 4. leaves, in index order */
    for (uint64_t i = 0; i < n; i++) {
        if (res[i].code != ORC_OK) continue;
        const orc_ept_map *m = &maps[i];
        uint64_t key = map_key(1, m->gpa);
        uint64_t *hit = nt ? (uint64_t *)bsearch(&key, keys, nt, sizeof(uint64_t), cmp_u64) : NULL;
        uint64_t pt = hit ? pool[hit - keys] : existing_ept_table(v, m->gpa, 1);
        store64(v->arena + ept_entry_off(pt, 1, m->gpa), m->hpa | (m->flags & 7u) | ORC_EPT_WB);
    }
    free(keys);
    return (int64_t)nt;
}

/* GPA -> arena offset through VM vm's EPT for an access that needs `need`
 * (bit 0 read, bit 1 write; 0: any present leaf), read-only: the walk the
 * copies use, exposed so that the effect of EPT maps can be checked. */
uint32_t orc_ept_xlat(const orc_state *s, uint32_t vm, uint64_t gpa, uint32_t need, uint64_t *hpa) {
    if (vm >= s->nvm || !s->vms[vm].has_ept) return ORC_INVALID;
    *hpa = 0;
    return ept_walk(&s->vms[vm], gpa, need, hpa, NULL);
}
