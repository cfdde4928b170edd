/*
 * thin_oracle.c -- plain, slow, sequential CPU oracle for the lambda-leveling
 * loop of grayscale topological thinning (the Couprie-Bertrand operator as
 * restated by Mahmoudi, Akil and Matas, "Parallel image thinning through
 * topological operators on shared memory parallel machines", section 2).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link,
 * load or call this file: only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, table or header
 * with the GPU library; the two meet only on seeded synthetic inputs.
 *
 * Everything here is written from the definitions in section 2.1:
 *   - an image F maps pixels to integers; the section F_k is {x : F(x) >= k};
 *   - sections use n-adjacency and their complements n'-adjacency, with
 *     (n, n') = (8,4) or (4,8);
 *   - T(x, X) counts the n-components of the 8-ring of x inside X that are
 *     n-adjacent to x; a point is simple when T(x, X) = 1 and the same count
 *     taken for the complement with n' is 1 (the printed "= 0" for the
 *     complement is read as 1: the textbook characterisation);
 *   - x is destructible when it is simple for F_k with k = F(x);
 *   - Gamma+ (neighbours >= F(x)) and Gamma-- (neighbours < F(x)); the
 *     lowering target alpha- is max F over Gamma--, or F(x) when it is empty;
 *   - T+ = #C_n[x, Gamma+] and T-- = #C_n'[x, Gamma--] (the complement side
 *     uses n', so destructible <=> T+ = 1 and T-- = 1);
 *   - x is k-divergent when T-- = k > 1;
 *   - x is lambda-destructible when it is destructible, or k-divergent with at
 *     least k-1 of the counted lower components c satisfying
 *     F(x) - m(c) <= lambda;
 *   - x is a peak point when T+ = 0, and lambda-deletable when it is
 *     lambda-destructible, or a peak with F(x) - alpha- <= lambda;
 *   - x is an end point (for F) when exactly one of its n-neighbours lies in
 *     the section F_k, k = F(x), and a lambda-end point when it is an end
 *     point with F(x) - alpha- > lambda.
 *
 * Two operators, both "lower a point of the type set to alpha- until
 * stability" (section 2.2), differ only in the type set:
 *   op 0, lambda-leveling: the lambda-destructible points;
 *   op 1, lambda-skeleton (the algorithm box of section 2.2): the points that
 *         are lambda-deletable and not lambda-end.
 *
 * Readings of points the paper leaves open (listed with reasons in the design
 * notes of the repository):
 *   - m(c), the paper's undefined F^-(c), is read as the maximum of F over
 *     the pixels of c (the same contrast measure, F(x) - alpha-, the paper
 *     uses for peaks and lambda-end points).  PARITY UNPINNED: the paper
 *     prints no example that separates this from other readings; the tests
 *     pin every part of the predicate that does not depend on it (lambda = 0,
 *     lambda at or above the value range, and the section invariants).
 *   - The 1-pixel frame of the image is read-only (F is defined on Z^2 in the
 *     paper; a finite image needs a border rule).  Images with fewer than 3
 *     rows or columns have no interior and are returned unchanged.
 *   - The removal order (the paper selects "a point of minimal value" without
 *     a tie-break) is fixed as a sweep of the four parity classes
 *     (i mod 2, j mod 2) = (0,0), (0,1), (1,0), (1,1), each visited in raster
 *     order.  Two pixels of one class are never 8-adjacent, so lowering a
 *     class pixel by pixel equals lowering it all at once.  A separate queue
 *     oracle follows the paper's own minimal-value order for invariant checks.
 *   - One visit lowers a point at most once, to alpha- (the algorithm box of
 *     section 2.2 assigns F(x) := alpha- once per selection).
 *   - "Until stability" ends after a full four-class pass with no lowering;
 *     the pass count P includes that final pass.
 *
 * Pixels are held as int32 here (F: Z^2 -> Z); callers convert u8/u16.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* The 8-ring of x in a fixed order: E, NE, N, NW, W, SW, S, SE.
 * Row offset di (row i grows downward) and column offset dj. */
static const int RING_DI[8] = {0, -1, -1, -1, 0, 1, 1, 1};
static const int RING_DJ[8] = {1, 1, 0, -1, -1, -1, 0, 1};

static int iabs(int a) { return a < 0 ? -a : a; }

/* Adjacency of two offsets (a != b) in the sense of section 2.1:
 * 4-adjacent when |d1| + |d2| <= 1, 8-adjacent when max(|d1|, |d2|) <= 1. */
static int offsets_adjacent(int di, int dj, int m)
{
    if (di == 0 && dj == 0) return 0;
    if (m == 4) return iabs(di) + iabs(dj) <= 1;
    return iabs(di) <= 1 && iabs(dj) <= 1;
}

/* Components of the ring subset {p : member[p]} under m-adjacency, computed
 * by flood fill using only ring pixels (paths never pass through x).
 * label[p] receives a component id (0..) for members and -1 otherwise.
 * Returns the number of components. */
static int ring_components(const int member[8], int m, int label[8])
{
    int ncomp = 0;
    for (int p = 0; p < 8; ++p) label[p] = -1;
    for (int seed = 0; seed < 8; ++seed) {
        if (!member[seed] || label[seed] >= 0) continue;
        int stack[8], top = 0;
        stack[top++] = seed;
        label[seed] = ncomp;
        while (top > 0) {
            int a = stack[--top];
            for (int b = 0; b < 8; ++b) {
                if (!member[b] || label[b] >= 0) continue;
                if (offsets_adjacent(RING_DI[b] - RING_DI[a], RING_DJ[b] - RING_DJ[a], m)) {
                    label[b] = ncomp;
                    stack[top++] = b;
                }
            }
        }
        ++ncomp;
    }
    return ncomp;
}

/* Marks which components are counted in #C_m[x, .]: those holding at least
 * one pixel m-adjacent to x.  Returns how many are counted. */
static int counted_components(const int label[8], int ncomp, int m, int counted[8])
{
    int k = 0;
    for (int c = 0; c < 8; ++c) counted[c] = 0;
    for (int p = 0; p < 8; ++p)
        if (label[p] >= 0 && offsets_adjacent(RING_DI[p], RING_DJ[p], m))
            counted[label[p]] = 1;
    for (int c = 0; c < ncomp; ++c) k += counted[c];
    return k;
}

/* Result of characterising one point from its 3x3 neighbourhood. */
typedef struct {
    int32_t tplus;          /* T+  = #C_n [x, Gamma+]                        */
    int32_t tminus;         /* T-- = #C_n'[x, Gamma--]  (= k)                */
    int32_t destructible;   /* T+ = 1 and T-- = 1                           */
    int32_t lambda_destr;   /* lambda-destructible                          */
    int64_t alpha_minus;    /* max over Gamma--, or F(x) if empty           */
    int64_t comp_max[4];    /* m(c) of each counted lower component, in    */
                            /* order of first ring position; unused = -1    */
    int32_t qualifying;     /* #counted components with F(x) - m(c) <= lam  */
    int32_t peak;           /* T+ = 0                                       */
    int32_t end;            /* exactly one n-neighbour y with F(y) >= F(x)  */
    int32_t lambda_deletable; /* lambda-destructible, or a peak with        */
                            /* F(x) - alpha- <= lambda                      */
    int32_t lambda_end;     /* end point with F(x) - alpha- > lambda        */
    int32_t skeleton;       /* lambda-deletable and not lambda-end          */
    int32_t pad;
} oracle_point;

/* adjacency: 0 = (8,4), 1 = (4,8). nb[p] = F at ring position p. */
void oracle_classify(const int64_t nb[8], int64_t v, int32_t adjacency, uint32_t lambda,
                     oracle_point* out)
{
    const int n = adjacency == 0 ? 8 : 4;
    const int nbar = adjacency == 0 ? 4 : 8;
    int upper[8], lower[8], lab_u[8], lab_l[8], cnt_u[8], cnt_l[8];
    for (int p = 0; p < 8; ++p) {
        upper[p] = nb[p] >= v;  /* Gamma+  */
        lower[p] = nb[p] < v;   /* Gamma-- */
    }
    int ncu = ring_components(upper, n, lab_u);
    int ncl = ring_components(lower, nbar, lab_l);
    out->tplus = counted_components(lab_u, ncu, n, cnt_u);
    out->tminus = counted_components(lab_l, ncl, nbar, cnt_l);
    out->destructible = (out->tplus == 1 && out->tminus == 1);

    /* alpha-: highest strictly lower neighbour, over all of Gamma--. */
    out->alpha_minus = v;
    int any_lower = 0;
    for (int p = 0; p < 8; ++p)
        if (lower[p]) {
            if (!any_lower || nb[p] > out->alpha_minus) out->alpha_minus = nb[p];
            any_lower = 1;
        }

    /* m(c) for each counted lower component, listed by component id. */
    for (int i = 0; i < 4; ++i) out->comp_max[i] = -1;
    int slot = 0;
    out->qualifying = 0;
    for (int c = 0; c < ncl; ++c) {
        if (!cnt_l[c]) continue;
        int64_t m = -1;
        for (int p = 0; p < 8; ++p)
            if (lab_l[p] == c && nb[p] > m) m = nb[p];
        if (slot < 4) out->comp_max[slot] = m;
        ++slot;
        if (v - m <= (int64_t)lambda) out->qualifying += 1;
    }
    const int k = out->tminus;
    out->lambda_destr = out->destructible || (k > 1 && out->qualifying >= k - 1);

    /* Peak and end points, and the skeleton's type set.  The contrast
     * F(x) - alpha- is 0 when Gamma-- is empty (alpha- = F(x) then). */
    const int64_t contrast = v - out->alpha_minus;
    int upper_n_neighbours = 0;
    for (int p = 0; p < 8; ++p)
        if (upper[p] && offsets_adjacent(RING_DI[p], RING_DJ[p], n)) ++upper_n_neighbours;
    out->peak = out->tplus == 0;
    out->end = upper_n_neighbours == 1;
    out->lambda_deletable = out->lambda_destr || (out->peak && contrast <= (int64_t)lambda);
    out->lambda_end = out->end && contrast > (int64_t)lambda;
    out->skeleton = out->lambda_deletable && !out->lambda_end;
    out->pad = 0;
}

/* Whether operator `op` lowers a characterised point (section 2.2: op 0 the
 * lambda-destructible type set, op 1 the lambda-skeleton's). */
static int lowerable(const oracle_point* pt, int32_t op)
{
    return op == 1 ? pt->skeleton : pt->lambda_destr;
}

/* Characterise interior pixel (i, j) of F (row-major, h x w). */
static void classify_at(const int32_t* F, int64_t w, int64_t i, int64_t j, int32_t adjacency,
                        uint32_t lambda, oracle_point* out)
{
    int64_t nb[8];
    for (int p = 0; p < 8; ++p) nb[p] = F[(i + RING_DI[p]) * w + (j + RING_DJ[p])];
    oracle_classify(nb, F[i * w + j], adjacency, lambda, out);
}

/* Parity classes in sweep order: (i mod 2, j mod 2). */
static const int CLASS_I[4] = {0, 0, 1, 1};
static const int CLASS_J[4] = {0, 1, 0, 1};

enum { ORACLE_OK = 0, ORACLE_EINVAL = -1, ORACLE_ENOMEM = -2, ORACLE_ELIMIT = -4 };

/*
 * ORACLE-SWEEP: lower the points of operator op's type set (op 0 the
 * lambda-destructible points, op 1 the lambda-skeleton's) until stability,
 * visiting the four parity classes in order, each in raster order, every
 * interior pixel of the class once per visit.
 * max_passes = 0 means no cap; when the cap is reached before stability the
 * function returns ORACLE_ELIMIT with F holding the state after the last pass.
 * passes_out: passes run, including the final pass without any lowering.
 */
int oracle_sweep(int32_t* F, int64_t h, int64_t w, uint32_t lambda, int32_t adjacency,
                 int32_t op, uint64_t max_passes, uint64_t* passes_out, uint64_t* lowerings_out)
{
    if (h < 0 || w < 0 || (adjacency != 0 && adjacency != 1) || (op != 0 && op != 1))
        return ORACLE_EINVAL;
    uint64_t passes = 0, lowerings = 0;
    int status = ORACLE_OK;
    if (h >= 3 && w >= 3) {
        for (;;) {
            if (max_passes && passes == max_passes) { status = ORACLE_ELIMIT; break; }
            uint64_t lowered_this_pass = 0;
            for (int s = 0; s < 4; ++s) {
                for (int64_t i = 1; i < h - 1; ++i) {
                    if ((i & 1) != CLASS_I[s]) continue;
                    for (int64_t j = 1; j < w - 1; ++j) {
                        if ((j & 1) != CLASS_J[s]) continue;
                        oracle_point pt;
                        classify_at(F, w, i, j, adjacency, lambda, &pt);
                        if (lowerable(&pt, op)) {
                            F[i * w + j] = (int32_t)pt.alpha_minus;
                            ++lowered_this_pass;
                        }
                    }
                }
            }
            ++passes;
            lowerings += lowered_this_pass;
            if (lowered_this_pass == 0) break;
        }
    }
    if (passes_out) *passes_out = passes;
    if (lowerings_out) *lowerings_out = lowerings;
    return status;
}

/*
 * Same sweep, but the pixels of each class may be visited in any order given
 * by `order` (a permutation of 0..h*w-1; entries that are not interior pixels
 * of the class being visited are skipped).  Lowering one class pixel by pixel
 * in any order must give the raster-order result bit for bit.
 */
int oracle_sweep_ordered(int32_t* F, int64_t h, int64_t w, uint32_t lambda, int32_t adjacency,
                         int32_t op, const int64_t* order, uint64_t* passes_out,
                         uint64_t* lowerings_out)
{
    if (h < 0 || w < 0 || (adjacency != 0 && adjacency != 1) || (op != 0 && op != 1) || !order)
        return ORACLE_EINVAL;
    uint64_t passes = 0, lowerings = 0;
    if (h >= 3 && w >= 3) {
        for (;;) {
            uint64_t lowered_this_pass = 0;
            for (int s = 0; s < 4; ++s) {
                for (int64_t t = 0; t < h * w; ++t) {
                    int64_t i = order[t] / w, j = order[t] % w;
                    if (i < 1 || i > h - 2 || j < 1 || j > w - 2) continue;
                    if ((i & 1) != CLASS_I[s] || (j & 1) != CLASS_J[s]) continue;
                    oracle_point pt;
                    classify_at(F, w, i, j, adjacency, lambda, &pt);
                    if (lowerable(&pt, op)) {
                        F[i * w + j] = (int32_t)pt.alpha_minus;
                        ++lowered_this_pass;
                    }
                }
            }
            ++passes;
            lowerings += lowered_this_pass;
            if (lowered_this_pass == 0) break;
        }
    }
    if (passes_out) *passes_out = passes;
    if (lowerings_out) *lowerings_out = lowerings;
    return ORACLE_OK;
}

/*
 * ORACLE-SWEEP-DIRTY: the same sweep, visiting in each class only the pixels
 * that may have changed status: a pixel's decision is a function of its 3x3
 * neighbourhood, so it is re-examined only after it or one of its eight
 * neighbours was lowered (the re-examination rule of section 2.2).  Output,
 * pass count and lowering count equal ORACLE-SWEEP's; examinations_out counts
 * the characterisations actually performed.
 */
int oracle_sweep_dirty(int32_t* F, int64_t h, int64_t w, uint32_t lambda, int32_t adjacency,
                       int32_t op, uint64_t* passes_out, uint64_t* lowerings_out,
                       uint64_t* examinations_out)
{
    if (h < 0 || w < 0 || (adjacency != 0 && adjacency != 1) || (op != 0 && op != 1))
        return ORACLE_EINVAL;
    uint64_t lowerings = 0, exams = 0, passes = 0;
    if (h >= 3 && w >= 3) {
        const int64_t npix = h * w;
        uint8_t* pending = (uint8_t*)calloc((size_t)npix, 1);
        int64_t* list[4];
        int64_t len[4] = {0, 0, 0, 0};
        int64_t* next = (int64_t*)malloc(sizeof(int64_t) * (size_t)npix);
        for (int s = 0; s < 4; ++s) list[s] = (int64_t*)malloc(sizeof(int64_t) * (size_t)npix);
        if (!pending || !next || !list[0] || !list[1] || !list[2] || !list[3]) {
            free(pending); free(next);
            for (int s = 0; s < 4; ++s) free(list[s]);
            return ORACLE_ENOMEM;
        }
        /* Class index of pixel (i, j) in sweep order. */
#define CLASS_OF(i, j) ((int)(((i) & 1) * 2 + ((j) & 1)))
        for (int64_t i = 1; i < h - 1; ++i)
            for (int64_t j = 1; j < w - 1; ++j) {
                int s = CLASS_OF(i, j);
                list[s][len[s]++] = i * w + j;
                pending[i * w + j] = 1;
            }
        int64_t step = 0, last_lowering_step = -1;
        int idle_steps = 0;
        while (idle_steps < 4) {
            int s = (int)(step & 3);
            /* Snapshot this class's pending list; pixels of the same class
             * that become pending during the visit wait for the next visit. */
            int64_t n = len[s];
            memcpy(next, list[s], sizeof(int64_t) * (size_t)n);
            len[s] = 0;
            for (int64_t t = 0; t < n; ++t) pending[next[t]] = 0;
            int lowered_any = 0;
            for (int64_t t = 0; t < n; ++t) {
                int64_t idx = next[t], i = idx / w, j = idx % w;
                oracle_point pt;
                classify_at(F, w, i, j, adjacency, lambda, &pt);
                ++exams;
                if (!lowerable(&pt, op)) continue;
                F[idx] = (int32_t)pt.alpha_minus;
                ++lowerings;
                lowered_any = 1;
                for (int di = -1; di <= 1; ++di)
                    for (int dj = -1; dj <= 1; ++dj) {
                        int64_t a = i + di, b = j + dj;
                        if (a < 1 || a > h - 2 || b < 1 || b > w - 2) continue;
                        if (pending[a * w + b]) continue;
                        int c = CLASS_OF(a, b);
                        pending[a * w + b] = 1;
                        list[c][len[c]++] = a * w + b;
                    }
            }
            if (lowered_any) { last_lowering_step = step; idle_steps = 0; }
            else ++idle_steps;
            ++step;
        }
#undef CLASS_OF
        /* Passes: the pass holding the last lowering, plus the final pass
         * without change; a single pass when nothing was ever lowered. */
        passes = last_lowering_step < 0 ? 1 : (uint64_t)(last_lowering_step / 4) + 2;
        free(pending); free(next);
        for (int s = 0; s < 4; ++s) free(list[s]);
    }
    if (passes_out) *passes_out = passes;
    if (lowerings_out) *lowerings_out = lowerings;
    if (examinations_out) *examinations_out = exams;
    return ORACLE_OK;
}

/*
 * ORACLE-QUEUE: the sequential algorithm of section 2.2 with operator op's
 * type set: repeatedly select a point of the type set of minimal value and
 * lower it to alpha-, re-examining the eight neighbours of every lowered
 * point (every point of the type set is queued: it was queued at the start
 * or when its 3x3 last changed, so the first one popped is a minimal one).  A binary min-heap keyed (F(x), i, j) holds the points
 * to examine; a point is never queued twice.  Only the popped point changes,
 * so the keys of queued points never go stale.  Results depend on the order
 * and are compared with the sweep by invariants only.
 */
typedef struct { int64_t key; int64_t idx; } heap_item;

static int heap_less(const heap_item* a, const heap_item* b)
{
    return a->key < b->key || (a->key == b->key && a->idx < b->idx);
}

static void heap_push(heap_item* hp, int64_t* n, heap_item it)
{
    int64_t c = (*n)++;
    hp[c] = it;
    while (c > 0) {
        int64_t p = (c - 1) / 2;
        if (!heap_less(&hp[c], &hp[p])) break;
        heap_item tmp = hp[p]; hp[p] = hp[c]; hp[c] = tmp;
        c = p;
    }
}

static heap_item heap_pop(heap_item* hp, int64_t* n)
{
    heap_item top = hp[0];
    hp[0] = hp[--(*n)];
    int64_t c = 0;
    for (;;) {
        int64_t l = 2 * c + 1, r = l + 1, m = c;
        if (l < *n && heap_less(&hp[l], &hp[m])) m = l;
        if (r < *n && heap_less(&hp[r], &hp[m])) m = r;
        if (m == c) break;
        heap_item tmp = hp[m]; hp[m] = hp[c]; hp[c] = tmp;
        c = m;
    }
    return top;
}

int oracle_queue(int32_t* F, int64_t h, int64_t w, uint32_t lambda, int32_t adjacency,
                 int32_t op, uint64_t* lowerings_out, uint64_t* pops_out)
{
    if (h < 0 || w < 0 || (adjacency != 0 && adjacency != 1) || (op != 0 && op != 1))
        return ORACLE_EINVAL;
    uint64_t lowerings = 0, pops = 0;
    if (h >= 3 && w >= 3) {
        const int64_t npix = h * w;
        heap_item* hp = (heap_item*)malloc(sizeof(heap_item) * (size_t)npix);
        uint8_t* queued = (uint8_t*)calloc((size_t)npix, 1);
        if (!hp || !queued) { free(hp); free(queued); return ORACLE_ENOMEM; }
        int64_t n = 0;
        for (int64_t i = 1; i < h - 1; ++i)
            for (int64_t j = 1; j < w - 1; ++j) {
                heap_item it = {F[i * w + j], i * w + j};
                heap_push(hp, &n, it);
                queued[i * w + j] = 1;
            }
        while (n > 0) {
            heap_item it = heap_pop(hp, &n);
            ++pops;
            int64_t idx = it.idx, i = idx / w, j = idx % w;
            queued[idx] = 0;
            oracle_point pt;
            classify_at(F, w, i, j, adjacency, lambda, &pt);
            if (!lowerable(&pt, op)) continue;
            F[idx] = (int32_t)pt.alpha_minus;
            ++lowerings;
            for (int di = -1; di <= 1; ++di)
                for (int dj = -1; dj <= 1; ++dj) {
                    int64_t a = i + di, b = j + dj;
                    if (a < 1 || a > h - 2 || b < 1 || b > w - 2) continue;
                    if (queued[a * w + b]) continue;
                    heap_item nx = {F[a * w + b], a * w + b};
                    heap_push(hp, &n, nx);
                    queued[a * w + b] = 1;
                }
        }
        free(hp); free(queued);
    }
    if (lowerings_out) *lowerings_out = lowerings;
    if (pops_out) *pops_out = pops;
    return ORACLE_OK;
}

/* Number of interior pixels of F that are lambda-destructible (a stable
 * image has none) and, separately, the number that are destructible. */
int oracle_count_destructible(const int32_t* F, int64_t h, int64_t w, uint32_t lambda,
                              int32_t adjacency, uint64_t* lambda_destr_out,
                              uint64_t* destr_out)
{
    if (h < 0 || w < 0 || (adjacency != 0 && adjacency != 1)) return ORACLE_EINVAL;
    uint64_t ld = 0, d = 0;
    for (int64_t i = 1; i + 1 < h; ++i)
        for (int64_t j = 1; j + 1 < w; ++j) {
            oracle_point pt;
            classify_at(F, w, i, j, adjacency, lambda, &pt);
            ld += (uint64_t)pt.lambda_destr;
            d += (uint64_t)pt.destructible;
        }
    if (lambda_destr_out) *lambda_destr_out = ld;
    if (destr_out) *destr_out = d;
    return ORACLE_OK;
}

/* Number of interior pixels of F that operator `op` would lower (a stable
 * image has none). */
int oracle_count_lowerable(const int32_t* F, int64_t h, int64_t w, uint32_t lambda,
                           int32_t adjacency, int32_t op, uint64_t* count_out)
{
    if (h < 0 || w < 0 || (adjacency != 0 && adjacency != 1) || (op != 0 && op != 1))
        return ORACLE_EINVAL;
    uint64_t c = 0;
    for (int64_t i = 1; i + 1 < h; ++i)
        for (int64_t j = 1; j + 1 < w; ++j) {
            oracle_point pt;
            classify_at(F, w, i, j, adjacency, lambda, &pt);
            c += (uint64_t)lowerable(&pt, op);
        }
    if (count_out) *count_out = c;
    return ORACLE_OK;
}

/* Ring offsets, exported so tests can lay out 3x3 patches the same way. */
void oracle_ring_offsets(int32_t di[8], int32_t dj[8])
{
    for (int p = 0; p < 8; ++p) { di[p] = RING_DI[p]; dj[p] = RING_DJ[p]; }
}
