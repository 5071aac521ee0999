/*
 * Seeded input generation helpers (plain C, host only).
 *
 * This file belongs to the synthetic workload generator.  It holds none of
 * the translation or copy arithmetic; it only produces input bytes and a
 * request-to-epoch assignment, and both the CPU oracle's inputs and the GPU
 * library's inputs are built from its output.
 *
 *   wl_fill          closed-form byte fill: the 8-byte little-endian word at
 *                    byte offset 8*i of a buffer keyed (seed, key) equals
 *                    splitmix64(seed ^ (key << 48) ^ i), where splitmix64 is
 *                    Vigna's public-domain mixer (state += 0x9E3779B97F4A7C15,
 *                    then two xor-shift-multiply rounds and a final xor-shift).
 *   wl_assign_epochs greedy epoch cut: requests are taken in index order and a
 *                    new epoch starts whenever adding the next request would
 *                    push the bytes placed in its VMA past that VMA's budget.
 */
#include <stdint.h>
#include <string.h>
#include <pthread.h>

static inline uint64_t wl_mix(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

/* Fill dst[0..bytes) with the bytes at absolute offsets [off, off+bytes). */
static void fill_range(uint8_t *dst, uint64_t off, uint64_t bytes, uint64_t seed, uint64_t key) {
    uint64_t base = seed ^ (key << 48);
    uint64_t o = off, end = off + bytes;
    /* unaligned head */
    while (o < end && (o & 7)) {
        uint64_t w = wl_mix(base ^ (o >> 3));
        *dst++ = (uint8_t)(w >> (8 * (o & 7)));
        o++;
    }
    /* whole words */
    while (o + 8 <= end) {
        uint64_t w = wl_mix(base ^ (o >> 3));
        memcpy(dst, &w, 8);
        dst += 8;
        o += 8;
    }
    /* tail */
    while (o < end) {
        uint64_t w = wl_mix(base ^ (o >> 3));
        *dst++ = (uint8_t)(w >> (8 * (o & 7)));
        o++;
    }
}

typedef struct {
    uint8_t *dst;
    uint64_t off, bytes, seed, key;
} fill_job;

static void *fill_worker(void *p) {
    fill_job *j = (fill_job *)p;
    fill_range(j->dst, j->off, j->bytes, j->seed, j->key);
    return NULL;
}

int wl_fill(uint8_t *dst, uint64_t off, uint64_t bytes, uint64_t seed, uint64_t key, int nthreads) {
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    if (bytes < (16ull << 20) || nthreads == 1) {
        fill_range(dst, off, bytes, seed, key);
        return 0;
    }
    pthread_t th[64];
    fill_job jobs[64];
    uint64_t per = ((bytes / (uint64_t)nthreads) + 4095) & ~4095ull;
    int started = 0;
    uint64_t pos = 0;
    for (int t = 0; t < nthreads && pos < bytes; t++) {
        uint64_t n = per;
        if (pos + n > bytes) n = bytes - pos;
        jobs[t].dst = dst + pos;
        jobs[t].off = off + pos;
        jobs[t].bytes = n;
        jobs[t].seed = seed;
        jobs[t].key = key;
        if (pthread_create(&th[t], NULL, fill_worker, &jobs[t]) != 0) {
            fill_range(jobs[t].dst, jobs[t].off, jobs[t].bytes, seed, key);
            jobs[t].bytes = 0;
            th[t] = 0;
        }
        started = t + 1;
        pos += n;
    }
    for (int t = 0; t < started; t++)
        if (th[t]) pthread_join(th[t], NULL);
    return 0;
}

/*
 * Greedy epoch assignment.  vma[i] is the global VMA id request i lands in,
 * len[i] its length, budget[v] the bytes one epoch may place in VMA v.
 * used[] is scratch of nvma entries.  Writes epoch_end[] (exclusive request
 * index ending each epoch) and returns the number of epochs.
 */
uint64_t wl_assign_epochs(const uint32_t *vma, const uint64_t *len, uint64_t n,
                          const uint64_t *budget, uint64_t nvma, uint64_t *used,
                          uint64_t *epoch_end) {
    uint64_t ne = 0;
    /* touched[] lists the VMAs used in the current epoch so resetting is O(epoch) */
    memset(used, 0, nvma * sizeof(uint64_t));
    uint64_t start = 0;
    for (uint64_t i = 0; i < n; i++) {
        uint32_t v = vma[i];
        if (i > start && used[v] + len[i] > budget[v]) {
            epoch_end[ne++] = i;
            for (uint64_t k = start; k < i; k++) used[vma[k]] = 0;
            start = i;
        }
        used[v] += len[i];
    }
    if (n > 0) epoch_end[ne++] = n;
    return ne;
}
