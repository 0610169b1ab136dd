/*
 * rcm_oracle.c -- plain, slow, single-threaded CPU oracle for Reverse
 * Cuthill-McKee ordering (Azad, Jacquelin, Buluc, Ng, "The Reverse
 * Cuthill-McKee Algorithm in Distributed-Memory").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it.  It shares no code, header or
 * table with the GPU library; the status codes below are numerically equal to
 * the library's because both follow the same documented interface.
 *
 * What is computed, and where the paper defines it:
 *   - bandwidth and envelope size (profile) of a symmetric pattern:
 *     Section II-A definitions of f_i, beta_i, beta(A) and Env(A);
 *   - degrees: the dense vector D consumed by Algorithms 3 and 4;
 *   - pseudo-peripheral vertex: Algorithm 2 (George-Liu), with Algorithm 4's
 *     alternative return value as an option;
 *   - Cuthill-McKee labelling: Algorithm 1 (serial queue form) and, as a
 *     self-check, Algorithm 3 (level-synchronous SpMSpV over the
 *     (select2nd, min) semiring followed by SortPerm on
 *     (parent label, degree, vertex id), Section IV-B);
 *   - one ordering per connected component (Section III-B), then reversal
 *     (last line of Algorithm 1, return statement of Algorithm 3).
 *
 * Readings taken where the paper leaves a choice open (each also listed in
 * the design notes of the repository):
 *   R1  the "arbitrary" start vertex of a component is its lowest vertex id;
 *   R2  ties in "minimum degree" are broken by the lower vertex id;
 *   R3  by default the pseudo-peripheral vertex is the root of the last BFS
 *       (Algorithm 2); variant 1 returns the min-(degree, id) vertex of the
 *       last level of the last BFS (Algorithm 4); the level counter of
 *       Algorithm 4 is taken per BFS, so both run the same BFS sequence;
 *   R4  degree = number of off-diagonal entries of the row (self loops do
 *       not count; duplicate entries are a malformed input, always rejected);
 *   R5  within a level, vertices are ordered by (parent label, degree, id),
 *       the id being the caller's vertex id;
 *   R6  components are processed in increasing order of their lowest id and
 *       receive consecutive label ranges; reversal is per component by
 *       default (variant 1 reverses the whole label sequence);
 *   R7  bandwidth uses 0-based indices and treats the diagonal as present:
 *       beta_k = k - min(k, min new index of a neighbour of row k); the
 *       envelope condition is read as 0 < i - j <= beta_i, so the profile is
 *       the sum of beta_k, accumulated in 64 bits.
 *
 * Parity pins: the pinning tests check this file against closed forms
 * (paths, complete graphs, k x m grids), a library bandwidth routine,
 * brute-force minimum bandwidth on tiny graphs, a library BFS, and the
 * equivalence of the Algorithm 1 and Algorithm 3 labellings.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_INVALID_ARGUMENT 1
#define ORC_ERR_BAD_CSR 2
#define ORC_ERR_NOT_SYMMETRIC 3
#define ORC_ERR_OUT_OF_MEMORY 5

typedef struct {
    int64_t bandwidth_before;
    int64_t profile_before;
    int64_t bandwidth_after;
    int64_t profile_after;
    int64_t edges_traversed;
    int32_t num_components;
    int32_t pseudo_diameter;
    int32_t num_bfs;
    int32_t num_levels;
} orc_stats;

/* ------------------------------------------------------------------------ */
/* Input checks (interface preconditions, not part of the paper's method).  */
/* ------------------------------------------------------------------------ */

static int row_contains(const int32_t* rowptr, const int32_t* colidx, int32_t row, int32_t col)
{
    for (int32_t k = rowptr[row]; k < rowptr[row + 1]; ++k)
        if (colidx[k] == col) return 1;
    return 0;
}

/* Structural checks and duplicate entries always (reading R4: a pattern is a
 * set of positions, so a repeated position is a malformed input); symmetry
 * (the paper's RCM is defined for symmetric matrices, Section V matrix
 * suite) when full_check. */
int orc_validate(int32_t n, const int32_t* rowptr, const int32_t* colidx, int full_check)
{
    if (n < 0) return ORC_ERR_INVALID_ARGUMENT;
    if (n == 0) return ORC_OK;
    if (rowptr == NULL) return ORC_ERR_INVALID_ARGUMENT;
    if (rowptr[0] != 0) return ORC_ERR_BAD_CSR;
    for (int32_t i = 0; i < n; ++i)
        if (rowptr[i + 1] < rowptr[i]) return ORC_ERR_BAD_CSR;
    if (rowptr[n] > 0 && colidx == NULL) return ORC_ERR_INVALID_ARGUMENT;
    for (int32_t k = 0; k < rowptr[n]; ++k)
        if (colidx[k] < 0 || colidx[k] >= n) return ORC_ERR_BAD_CSR;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t a = rowptr[i]; a < rowptr[i + 1]; ++a)
            for (int32_t b = a + 1; b < rowptr[i + 1]; ++b)
                if (colidx[a] == colidx[b]) return ORC_ERR_BAD_CSR;
    if (!full_check) return ORC_OK;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t a = rowptr[i]; a < rowptr[i + 1]; ++a)
            if (!row_contains(rowptr, colidx, colidx[a], i)) return ORC_ERR_NOT_SYMMETRIC;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Degrees: the vector D of Algorithms 3 and 4 (reading R4).                */
/* ------------------------------------------------------------------------ */

void orc_degrees(int32_t n, const int32_t* rowptr, const int32_t* colidx, int32_t* deg)
{
    for (int32_t v = 0; v < n; ++v) {
        int32_t d = 0;
        for (int32_t k = rowptr[v]; k < rowptr[v + 1]; ++k)
            if (colidx[k] != v) ++d;
        deg[v] = d;
    }
}

/* ------------------------------------------------------------------------ */
/* Bandwidth and profile (Section II-A), of P A P^T for perm = new->old.    */
/* perm == NULL means the identity order.  Reading R7.                      */
/* ------------------------------------------------------------------------ */

int orc_bw_profile(int32_t n, const int32_t* rowptr, const int32_t* colidx, const int32_t* perm,
                   int64_t* bandwidth, int64_t* profile)
{
    int32_t* iperm = NULL;
    if (perm != NULL && n > 0) {
        iperm = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
        if (!iperm) return ORC_ERR_OUT_OF_MEMORY;
        for (int32_t k = 0; k < n; ++k) iperm[perm[k]] = k;
    }
    int64_t bw = 0, prof = 0;
    for (int32_t k = 0; k < n; ++k) {
        int32_t v = perm ? perm[k] : k;
        int32_t f = k; /* first (lowest) column index in row k; diagonal counts */
        for (int32_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
            int32_t j = iperm ? iperm[colidx[e]] : colidx[e];
            if (j < f) f = j;
        }
        int64_t beta = (int64_t)k - f;
        if (beta > bw) bw = beta;
        prof += beta;
    }
    free(iperm);
    *bandwidth = bw;
    *profile = prof;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Rooted level structure L(v) (Section II-A) by breadth-first search.      */
/* level[] must hold -1 for every vertex of the component on entry; on exit */
/* it holds the distance from root.  order[] receives the vertices level by */
/* level; *count their number.  Returns the eccentricity l(root).           */
/* ------------------------------------------------------------------------ */

int32_t orc_level_structure(const int32_t* rowptr, const int32_t* colidx, int32_t root,
                            int32_t* level, int32_t* order, int32_t* count)
{
    int32_t head = 0, tail = 0;
    level[root] = 0;
    order[tail++] = root;
    int32_t ecc = 0;
    while (head < tail) {
        int32_t u = order[head++];
        for (int32_t k = rowptr[u]; k < rowptr[u + 1]; ++k) {
            int32_t v = colidx[k];
            if (level[v] < 0) {
                level[v] = level[u] + 1;
                if (level[v] > ecc) ecc = level[v];
                order[tail++] = v;
            }
        }
    }
    *count = tail;
    return ecc;
}

/* Vertex of minimum degree in the last level, ties to the lower id (R2). */
static int32_t min_degree_in_last_level(const int32_t* deg, const int32_t* level,
                                        const int32_t* order, int32_t count, int32_t ecc)
{
    int32_t best = -1;
    for (int32_t i = 0; i < count; ++i) {
        int32_t v = order[i];
        if (level[v] != ecc) continue;
        if (best < 0 || deg[v] < deg[best] || (deg[v] == deg[best] && v < best)) best = v;
    }
    return best;
}

/* ------------------------------------------------------------------------ */
/* Pseudo-peripheral vertex, Algorithm 2 (George-Liu) from start vertex s.  */
/* variant 0: return the root of the last level structure (Algorithm 2).    */
/* variant 1: return the min-degree vertex of its last level (Algorithm 4). */
/* level[] must be -1 on the component on entry and is -1 again on exit.    */
/* ------------------------------------------------------------------------ */

int32_t orc_pseudo_peripheral(const int32_t* rowptr, const int32_t* colidx, const int32_t* deg,
                              int32_t s, int variant, int32_t* level, int32_t* order,
                              int32_t* nbfs_out, int32_t* comp_size_out)
{
    int32_t count = 0;
    int32_t r = s;
    int32_t ecc_r = orc_level_structure(rowptr, colidx, r, level, order, &count);
    int32_t nbfs = 1;
    int32_t nlvl = ecc_r - 1;
    int32_t last_pick = min_degree_in_last_level(deg, level, order, count, ecc_r);
    while (ecc_r > nlvl) {
        nlvl = ecc_r;
        int32_t v = last_pick; /* shrink the last level: min degree */
        for (int32_t i = 0; i < count; ++i) level[order[i]] = -1;
        ecc_r = orc_level_structure(rowptr, colidx, v, level, order, &count);
        ++nbfs;
        last_pick = min_degree_in_last_level(deg, level, order, count, ecc_r);
        r = v;
    }
    for (int32_t i = 0; i < count; ++i) level[order[i]] = -1;
    *nbfs_out = nbfs;
    *comp_size_out = count;
    return variant == 1 ? last_pick : r;
}

/* ------------------------------------------------------------------------ */
/* Cuthill-McKee labelling, Algorithm 1 (serial queue form).                */
/* label[] holds -1 for unlabelled vertices; the component gets labels      */
/* base, base+1, ...; cm[label] = vertex.  Returns the number labelled and  */
/* stores the number of levels in *nlevels.                                 */
/* ------------------------------------------------------------------------ */

typedef struct { int32_t key0, key1, v; } orc_tuple;

static int cmp_tuple(const void* a, const void* b)
{
    const orc_tuple* x = (const orc_tuple*)a;
    const orc_tuple* y = (const orc_tuple*)b;
    if (x->key0 != y->key0) return x->key0 < y->key0 ? -1 : 1;
    if (x->key1 != y->key1) return x->key1 < y->key1 ? -1 : 1;
    if (x->v != y->v) return x->v < y->v ? -1 : 1;
    return 0;
}

int32_t orc_cm_queue(const int32_t* rowptr, const int32_t* colidx, const int32_t* deg,
                     int32_t root, int32_t base, int32_t* label, int32_t* cm,
                     int32_t* nlevels)
{
    int32_t head = base, tail = base;
    label[root] = tail;       /* v_1 <- r */
    cm[tail++] = root;
    /* Level bookkeeping for the statistics only.  In queue order every
     * vertex of level d is processed before any vertex of level d+1, and all
     * of level d+1 has been numbered once the last vertex of level d is done,
     * so each time the head reaches the end of the current level, the
     * vertices numbered so far beyond it form the next level. */
    int32_t level_end = tail;
    int32_t levels = 1;
    orc_tuple* buf = NULL;
    int32_t cap = 0;
    while (head < tail) {
        if (head == level_end) {
            level_end = tail;
            ++levels;
        }
        int32_t u = cm[head++];
        int32_t d = rowptr[u + 1] - rowptr[u];
        if (d > cap) {
            cap = d;
            orc_tuple* nb = (orc_tuple*)realloc(buf, sizeof(orc_tuple) * (size_t)cap);
            if (!nb) { free(buf); return -1; }
            buf = nb;
        }
        /* find all the unnumbered neighbours of u ... */
        int32_t c = 0;
        for (int32_t k = rowptr[u]; k < rowptr[u + 1]; ++k) {
            int32_t v = colidx[k];
            if (v == u || label[v] >= 0) continue;
            buf[c].key0 = deg[v];
            buf[c].key1 = 0;
            buf[c].v = v;
            ++c;
        }
        /* ... and number them in increasing order of degree (then id, R2);
         * with none, buf may still be NULL, which qsort must not be given */
        if (c > 0) qsort(buf, (size_t)c, sizeof(orc_tuple), cmp_tuple);
        for (int32_t i = 0; i < c; ++i) {
            label[buf[i].v] = tail;
            cm[tail++] = buf[i].v;
        }
    }
    free(buf);
    if (nlevels) *nlevels = levels;
    return tail - base;
}

/* ------------------------------------------------------------------------ */
/* Cuthill-McKee labelling, Algorithm 3 (level-synchronous, matrix form).   */
/* Same contract as orc_cm_queue.  parent[] is scratch of size n holding    */
/* INT32_MAX on entry and on exit.                                           */
/* ------------------------------------------------------------------------ */

int32_t orc_cm_levelsync(const int32_t* rowptr, const int32_t* colidx, const int32_t* deg,
                         int32_t root, int32_t base, int32_t* label, int32_t* cm,
                         int32_t* parent, int32_t* nlevels)
{
    int32_t nv = base;
    label[root] = nv;      /* R[r] <- 0 (offset by the component base) */
    cm[nv++] = root;
    int32_t cur_b = base, cur_e = nv;  /* L_cur = cm[cur_b, cur_e) */
    int32_t levels = 1;
    orc_tuple* T = NULL;
    int32_t cap = 0;
    while (cur_e > cur_b) {
        /* SpMSpV over (select2nd, min): every unlabelled neighbour of the
         * frontier receives the minimum label among its frontier neighbours;
         * Select keeps only unlabelled vertices (R == -1).  The next frontier
         * is collected in cm[] after the current one. */
        int32_t nxt = cur_e;
        for (int32_t p = cur_b; p < cur_e; ++p) {
            int32_t u = cm[p];
            for (int32_t k = rowptr[u]; k < rowptr[u + 1]; ++k) {
                int32_t v = colidx[k];
                if (label[v] >= 0) continue;
                if (parent[v] == INT32_MAX) cm[nxt++] = v;
                if (label[u] < parent[v]) parent[v] = label[u];
            }
        }
        int32_t cnt = nxt - cur_e;
        if (cnt == 0) break;
        if (cnt > cap) {
            cap = cnt;
            orc_tuple* nt = (orc_tuple*)realloc(T, sizeof(orc_tuple) * (size_t)cap);
            if (!nt) { free(T); return -1; }
            T = nt;
        }
        /* SortPerm: tuples (parent label, degree, id), lexicographic */
        for (int32_t i = 0; i < cnt; ++i) {
            int32_t v = cm[cur_e + i];
            T[i].key0 = parent[v];
            T[i].key1 = deg[v];
            T[i].v = v;
        }
        qsort(T, (size_t)cnt, sizeof(orc_tuple), cmp_tuple);
        /* R_next + nv, then Set the labels of the new level */
        for (int32_t i = 0; i < cnt; ++i) {
            int32_t v = T[i].v;
            label[v] = nv + i;
            cm[nv + i] = v;
            parent[v] = INT32_MAX;
        }
        nv += cnt;
        cur_b = cur_e;
        cur_e = nv;
        ++levels;
    }
    free(T);
    if (nlevels) *nlevels = levels;
    return nv - base;
}

/* ------------------------------------------------------------------------ */
/* Level orders: the alternatives to per-level sorting that Section VI      */
/* names as future work.  The component is labelled level by level of the   */
/* level structure rooted at root; within a level the vertices follow       */
/*   by_degree 0: increasing id (no sort: the order of the frontier vector) */
/*   by_degree 1: increasing (degree, id) (one global sort at the end by    */
/*                (level, degree, id); the parent label is not a key).      */
/* level[] must be -1 on the component on entry and is -1 again on exit.    */
/* Same output contract as orc_cm_queue.                                     */
/* ------------------------------------------------------------------------ */

int32_t orc_cm_level_order(const int32_t* rowptr, const int32_t* colidx, const int32_t* deg,
                           int32_t root, int32_t base, int by_degree, int32_t* label,
                           int32_t* cm, int32_t* level, int32_t* order, int32_t* nlevels)
{
    int32_t count = 0;
    int32_t ecc = orc_level_structure(rowptr, colidx, root, level, order, &count);
    orc_tuple* T = (orc_tuple*)malloc(sizeof(orc_tuple) * (size_t)(count > 0 ? count : 1));
    if (!T) return -1;
    for (int32_t i = 0; i < count; ++i) {
        int32_t v = order[i];
        T[i].key0 = level[v];
        T[i].key1 = by_degree ? deg[v] : 0;
        T[i].v = v;
    }
    /* lexicographic (level, degree or 0, id): the SortPerm comparison with
     * the level in the parent label's place */
    qsort(T, (size_t)count, sizeof(orc_tuple), cmp_tuple);
    for (int32_t i = 0; i < count; ++i) {
        label[T[i].v] = base + i;
        cm[base + i] = T[i].v;
    }
    for (int32_t i = 0; i < count; ++i) level[order[i]] = -1;
    free(T);
    if (nlevels) *nlevels = ecc + 1;
    return count;
}

/* ------------------------------------------------------------------------ */
/* Whole ordering.                                                          */
/*   pp_variant   0 = Algorithm 2 root (default), 1 = Algorithm 4 pick      */
/*   reverse_mode 0 = reverse each component's block (default), 1 = global  */
/*   full_check   also reject asymmetric patterns                          */
/*   cm_mode      0 = Algorithm 1 queue, 1 = Algorithm 3 level-synchronous, */
/*                2 = level order by id, 3 = level order by (degree, id)    */
/* perm_out[k] = original vertex placed at position k (new -> old).         */
/* Optional per-component outputs (each of capacity n, may be NULL):        */
/*   comp_offset[c], comp_root[c], comp_nbfs[c], comp_levels[c].            */
/* ------------------------------------------------------------------------ */

int orc_rcm_ex(int32_t n, const int32_t* rowptr, const int32_t* colidx, int pp_variant,
               int reverse_mode, int full_check, int cm_mode, int32_t* perm_out,
               int32_t* iperm_out, orc_stats* st, int32_t* comp_offset, int32_t* comp_root,
               int32_t* comp_nbfs, int32_t* comp_levels)
{
    orc_stats local;
    memset(&local, 0, sizeof(local));
    int status = orc_validate(n, rowptr, colidx, full_check);
    if (status != ORC_OK) return status;
    if (n > 0 && perm_out == NULL) return ORC_ERR_INVALID_ARGUMENT;
    if (n == 0) {
        if (st) *st = local;
        return ORC_OK;
    }
    size_t N = (size_t)n;
    int32_t* deg = (int32_t*)malloc(sizeof(int32_t) * N);
    int32_t* label = (int32_t*)malloc(sizeof(int32_t) * N);
    int32_t* cm = (int32_t*)malloc(sizeof(int32_t) * N);
    int32_t* level = (int32_t*)malloc(sizeof(int32_t) * N);
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * N);
    int32_t* parent = (int32_t*)malloc(sizeof(int32_t) * N);
    if (!deg || !label || !cm || !level || !order || !parent) {
        free(deg); free(label); free(cm); free(level); free(order); free(parent);
        return ORC_ERR_OUT_OF_MEMORY;
    }
    orc_degrees(n, rowptr, colidx, deg);
    orc_bw_profile(n, rowptr, colidx, NULL, &local.bandwidth_before, &local.profile_before);
    for (int32_t v = 0; v < n; ++v) { label[v] = -1; level[v] = -1; parent[v] = INT32_MAX; }

    int32_t ncomp = 0;
    int32_t nv = 0;
    for (int32_t s = 0; s < n; ++s) {
        if (label[s] >= 0) continue;
        /* s is the lowest id of a new component (R1, R6) */
        int32_t nbfs = 0, csize = 0;
        int32_t r = orc_pseudo_peripheral(rowptr, colidx, deg, s, pp_variant, level, order,
                                          &nbfs, &csize);
        int32_t nlev = 0, got;
        if (cm_mode == 1)
            got = orc_cm_levelsync(rowptr, colidx, deg, r, nv, label, cm, parent, &nlev);
        else if (cm_mode == 2 || cm_mode == 3)
            got = orc_cm_level_order(rowptr, colidx, deg, r, nv, cm_mode == 3, label, cm, level,
                                     order, &nlev);
        else
            got = orc_cm_queue(rowptr, colidx, deg, r, nv, label, cm, &nlev);
        if (got < 0) {
            free(deg); free(label); free(cm); free(level); free(order); free(parent);
            return ORC_ERR_OUT_OF_MEMORY;
        }
        int64_t m_c = 0;
        for (int32_t t = nv; t < nv + got; ++t) m_c += deg[cm[t]];
        if (comp_offset) comp_offset[ncomp] = nv;
        if (comp_root) comp_root[ncomp] = r;
        if (comp_nbfs) comp_nbfs[ncomp] = nbfs;
        if (comp_levels) comp_levels[ncomp] = nlev;
        local.num_bfs += nbfs;
        local.num_levels += nlev;
        if (nlev - 1 > local.pseudo_diameter) local.pseudo_diameter = nlev - 1;
        /* the labelled BFS scans the component once more; a level order
         * reuses the search's last level structure, unless the root is
         * Algorithm 4's pick, whose level structure is one more BFS */
        int extra = (cm_mode == 2 || cm_mode == 3) ? (pp_variant == 1 ? 1 : 0) : 1;
        local.edges_traversed += (int64_t)(nbfs + extra) * m_c;
        /* reverse this component's block (return of Algorithm 3) */
        if (reverse_mode == 0)
            for (int32_t t = 0; t < got; ++t) perm_out[nv + t] = cm[nv + got - 1 - t];
        nv += got;
        ++ncomp;
    }
    if (reverse_mode == 1)
        for (int32_t t = 0; t < n; ++t) perm_out[t] = cm[n - 1 - t]; /* w_i = v_{n-i+1} */
    local.num_components = ncomp;
    orc_bw_profile(n, rowptr, colidx, perm_out, &local.bandwidth_after, &local.profile_after);
    if (iperm_out)
        for (int32_t k = 0; k < n; ++k) iperm_out[perm_out[k]] = k;
    if (st) *st = local;
    free(deg); free(label); free(cm); free(level); free(order); free(parent);
    return ORC_OK;
}

int orc_rcm(int32_t n, const int32_t* rowptr, const int32_t* colidx, int pp_variant,
            int reverse_mode, int full_check, int32_t* perm_out, int32_t* iperm_out,
            orc_stats* st)
{
    return orc_rcm_ex(n, rowptr, colidx, pp_variant, reverse_mode, full_check, 0, perm_out,
                      iperm_out, st, NULL, NULL, NULL, NULL);
}
