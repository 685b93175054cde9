/*
 * Oracle for the supernodal sparse Cholesky (LL^T) method of
 * "Taking advantage of hybrid systems for sparse direct solvers via
 * task-based runtimes" (Lacoste, Faverge, Ramet, Thibault, Bosilca).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, serial, FP64 CPU
 * implementation written for checking; it is used by the test-suite, by the
 * package's smoke check and by the benchmark's CPU-baseline leg, and by
 * nothing else.  It shares no code, header or table with the GPU library.
 *
 * Every step follows the paper's Section III (ordering, elimination tree,
 * symbolic factorization, blocking, amalgamation, vertical splitting, the
 * three-step "1D task": diagonal factorization, triangular solve on the
 * panel, right-looking updates of the facing panels through a temporary
 * buffer as in the CPU scheme of Section V-B).  Where the paper is silent
 * (the ordering heuristic, tie-breaks, amalgamation rule, split rule, block
 * boundaries, flop convention) the reading implemented here is the one
 * written next to each function.
 *
 * Conventions: 0-based indices, CSC input with sorted rows, permutation
 * arrays are "new -> old" unless named iperm.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

typedef int32_t i32;
typedef int64_t i64;

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ENOTPD (-5)

static int cmp_i32(const void* a, const void* b)
{
    i32 x = *(const i32*)a, y = *(const i32*)b;
    return (x > y) - (x < y);
}

/* ------------------------------------------------------------------ */
/* O1. Graph of A + A^T without the diagonal (Section III: the solver  */
/* works on the symmetrized pattern).  Adjacency lists sorted, unique. */
/* adj must hold 2*nnz entries.  Returns the number of edges stored.   */
/* ------------------------------------------------------------------ */
i64 orc_graph(i32 n, const i64* colptr, const i32* rowind, i64* xadj, i32* adj)
{
    i64* deg = (i64*)calloc((size_t)n + 1, sizeof(i64));
    i64* fill = (i64*)malloc(((size_t)n + 1) * sizeof(i64));
    if (!deg || !fill) { free(deg); free(fill); return ORC_ENOMEM; }
    for (i32 j = 0; j < n; j++)
        for (i64 p = colptr[j]; p < colptr[j + 1]; p++) {
            i32 i = rowind[p];
            if (i < 0 || i >= n) { free(deg); free(fill); return ORC_EINVAL; }
            if (i != j) { deg[i]++; deg[j]++; }
        }
    xadj[0] = 0;
    for (i32 v = 0; v < n; v++) xadj[v + 1] = xadj[v] + deg[v];
    for (i32 v = 0; v <= n; v++) fill[v] = xadj[v];
    for (i32 j = 0; j < n; j++)
        for (i64 p = colptr[j]; p < colptr[j + 1]; p++) {
            i32 i = rowind[p];
            if (i != j) { adj[fill[i]++] = j; adj[fill[j]++] = i; }
        }
    i64 out = 0, lo = 0;
    for (i32 v = 0; v < n; v++) {
        i64 hi = xadj[v + 1];
        qsort(adj + lo, (size_t)(hi - lo), sizeof(i32), cmp_i32);
        i64 start = out;
        for (i64 p = lo; p < hi; p++)
            if (p == lo || adj[p] != adj[p - 1]) adj[out++] = adj[p];
        xadj[v] = start;
        lo = hi;
    }
    xadj[n] = out;
    free(deg);
    free(fill);
    return out;
}

/* ------------------------------------------------------------------ */
/* O2. Nested dissection (Section III: "nested dissection ... graph     */
/* partitioning", computed by Scotch in the paper).  Our pattern-only   */
/* reading, recursive on a vertex set C:                                */
/*   components of G[C] in ascending order of their smallest vertex;    */
/*   a component of size <= leaf is emitted in ascending id;            */
/*   otherwise a pseudo-peripheral root r is found (start at the        */
/*   smallest id; x = argmin (degree inside the component, id) over the */
/*   last BFS level; move to x while its eccentricity is larger), the   */
/*   level m is the first whose cumulative size reaches ceil(|C|/2)     */
/*   (m = e-1 if it is the last level e), the separator is the set of   */
/*   level-m vertices with a neighbour in level m+1; the rest is        */
/*   ordered recursively, then the separator in ascending id.           */
/* ------------------------------------------------------------------ */
typedef struct {
    i32 n;
    const i64* xadj;
    const i32* adj;
    i32 leaf;
    i32* tag;
    i32 ntag;
    i32* seen;
    i32 stamp;
    i32* level;
    i32* queue;
    i32* out;
    i32 nout;
    int err;
} nd_ctx;

/* BFS inside the vertices whose tag is tg; returns the eccentricity. */
static i32 nd_bfs(nd_ctx* c, i32 tg, i32 root)
{
    i32 st = ++c->stamp;
    i32 head = 0, tail = 0, ecc = 0;
    c->queue[tail++] = root;
    c->seen[root] = st;
    c->level[root] = 0;
    while (head < tail) {
        i32 v = c->queue[head++];
        for (i64 p = c->xadj[v]; p < c->xadj[v + 1]; p++) {
            i32 u = c->adj[p];
            if (c->tag[u] == tg && c->seen[u] != st) {
                c->seen[u] = st;
                c->level[u] = c->level[v] + 1;
                if (c->level[u] > ecc) ecc = c->level[u];
                c->queue[tail++] = u;
            }
        }
    }
    return ecc;
}

static void nd_emit_sorted(nd_ctx* c, i32* v, i32 cnt)
{
    qsort(v, (size_t)cnt, sizeof(i32), cmp_i32);
    for (i32 i = 0; i < cnt; i++) c->out[c->nout++] = v[i];
}

static void nd_rec(nd_ctx* c, i32* verts, i32 cnt);

static void nd_component(nd_ctx* c, i32* D, i32 d, i32 ctg)
{
    if (d <= c->leaf) { nd_emit_sorted(c, D, d); return; }
    i32 r = D[0];
    for (i32 i = 1; i < d; i++) if (D[i] < r) r = D[i];
    i32 e = nd_bfs(c, ctg, r);
    for (;;) {
        i32 x = -1, xdeg = 0;
        for (i32 i = 0; i < d; i++) {
            i32 v = D[i];
            if (c->level[v] != e) continue;
            i32 dg = 0;
            for (i64 p = c->xadj[v]; p < c->xadj[v + 1]; p++) if (c->tag[c->adj[p]] == ctg) dg++;
            if (x < 0 || dg < xdeg || (dg == xdeg && v < x)) { x = v; xdeg = dg; }
        }
        i32 ex = nd_bfs(c, ctg, x);
        if (ex > e) { r = x; e = ex; continue; }
        break;
    }
    e = nd_bfs(c, ctg, r); /* levels from the final root */
    i32* cnt = (i32*)calloc((size_t)e + 2, sizeof(i32));
    for (i32 i = 0; i < d; i++) cnt[c->level[D[i]]]++;
    i32 half = (d + 1) / 2, acc = 0, m = 0;
    for (m = 0; m <= e; m++) { acc += cnt[m]; if (acc >= half) break; }
    if (m == e) m = e - 1;
    free(cnt);
    i32* S = (i32*)malloc(sizeof(i32) * (size_t)d);
    i32* rest = (i32*)malloc(sizeof(i32) * (size_t)d);
    i32 ns = 0, nr = 0;
    for (i32 i = 0; i < d; i++) {
        i32 v = D[i];
        int sep = 0;
        if (c->level[v] == m)
            for (i64 p = c->xadj[v]; p < c->xadj[v + 1]; p++) {
                i32 u = c->adj[p];
                if (c->tag[u] == ctg && c->level[u] == m + 1) { sep = 1; break; }
            }
        if (sep) S[ns++] = v; else rest[nr++] = v;
    }
    nd_rec(c, rest, nr);
    nd_emit_sorted(c, S, ns);
    free(S);
    free(rest);
}

static void nd_rec(nd_ctx* c, i32* verts, i32 cnt)
{
    if (cnt == 0) return;
    i32 tg = ++c->ntag;
    for (i32 i = 0; i < cnt; i++) c->tag[verts[i]] = tg;
    qsort(verts, (size_t)cnt, sizeof(i32), cmp_i32);
    i32* comp = (i32*)malloc(sizeof(i32) * (size_t)cnt);
    i32* cstart = (i32*)malloc(sizeof(i32) * ((size_t)cnt + 1));
    i32* ctag = (i32*)malloc(sizeof(i32) * ((size_t)cnt + 1));
    i32 ncomp = 0, pos = 0;
    for (i32 i = 0; i < cnt; i++) {
        i32 s = verts[i];
        if (c->tag[s] != tg) continue;
        i32 ct = ++c->ntag;
        cstart[ncomp] = pos;
        ctag[ncomp] = ct;
        ncomp++;
        i32 head = pos;
        comp[pos++] = s;
        c->tag[s] = ct;
        while (head < pos) {
            i32 v = comp[head++];
            for (i64 p = c->xadj[v]; p < c->xadj[v + 1]; p++) {
                i32 u = c->adj[p];
                if (c->tag[u] == tg) { c->tag[u] = ct; comp[pos++] = u; }
            }
        }
    }
    cstart[ncomp] = pos;
    for (i32 k = 0; k < ncomp; k++)
        nd_component(c, comp + cstart[k], cstart[k + 1] - cstart[k], ctag[k]);
    free(comp);
    free(cstart);
    free(ctag);
}

/* order[new] = old vertex. */
int orc_nd(i32 n, const i64* xadj, const i32* adj, i32 leaf, i32* order)
{
    nd_ctx c;
    memset(&c, 0, sizeof(c));
    c.n = n; c.xadj = xadj; c.adj = adj; c.leaf = leaf < 1 ? 1 : leaf;
    c.tag = (i32*)calloc((size_t)n + 1, sizeof(i32));
    c.seen = (i32*)calloc((size_t)n + 1, sizeof(i32));
    c.level = (i32*)calloc((size_t)n + 1, sizeof(i32));
    c.queue = (i32*)malloc(sizeof(i32) * ((size_t)n + 1));
    i32* all = (i32*)malloc(sizeof(i32) * ((size_t)n + 1));
    if (!c.tag || !c.seen || !c.level || !c.queue || !all) return ORC_ENOMEM;
    for (i32 i = 0; i < n; i++) all[i] = i;
    c.out = order;
    nd_rec(&c, all, n);
    free(all); free(c.tag); free(c.seen); free(c.level); free(c.queue);
    return c.nout == n ? ORC_OK : ORC_EINVAL;
}

/* ------------------------------------------------------------------ */
/* O3/O4 (part). Elimination tree (Section III, [r87]) and column       */
/* counts of P A P^T for the ordering perm (new -> old), straight from  */
/* the definition of the symbolic factorization:                        */
/*   struct(L_{*,j}) = {i > j : a_ij != 0} U (U_{children c} struct(L_{*,c}) \ {j}) */
/*   parent(j) = min struct(L_{*,j}) \ {j}, -1 if empty;                */
/*   eta_j = |struct(L_{*,j})| counting the diagonal.                   */
/* The structures of children are dropped once merged.                  */
/* ------------------------------------------------------------------ */
int orc_etree_counts(i32 n, const i64* xadj, const i32* adj, const i32* perm, i32* parent, i64* eta)
{
    i32* iperm = (i32*)malloc(sizeof(i32) * ((size_t)n + 1));
    i32* mark = (i32*)malloc(sizeof(i32) * ((size_t)n + 1));
    i32** st = (i32**)calloc((size_t)n + 1, sizeof(i32*));
    i32* stlen = (i32*)calloc((size_t)n + 1, sizeof(i32));
    i32* head = (i32*)malloc(sizeof(i32) * ((size_t)n + 1));
    i32* next = (i32*)malloc(sizeof(i32) * ((size_t)n + 1));
    i32* buf = (i32*)malloc(sizeof(i32) * ((size_t)n + 1));
    if (!iperm || !mark || !st || !stlen || !head || !next || !buf) return ORC_ENOMEM;
    for (i32 k = 0; k < n; k++) { iperm[perm[k]] = k; mark[k] = -1; head[k] = -1; }
    for (i32 j = 0; j < n; j++) {
        i32 len = 0, mn = n;
        i32 oj = perm[j];
        for (i64 p = xadj[oj]; p < xadj[oj + 1]; p++) {
            i32 i = iperm[adj[p]];
            if (i > j && mark[i] != j) { mark[i] = j; buf[len++] = i; if (i < mn) mn = i; }
        }
        for (i32 ch = head[j]; ch >= 0; ch = next[ch]) {
            for (i32 q = 0; q < stlen[ch]; q++) {
                i32 i = st[ch][q];
                if (i != j && mark[i] != j) { mark[i] = j; buf[len++] = i; if (i < mn) mn = i; }
            }
            free(st[ch]);
            st[ch] = NULL;
        }
        eta[j] = (i64)len + 1;
        parent[j] = len ? mn : -1;
        if (len) {
            st[j] = (i32*)malloc(sizeof(i32) * (size_t)len);
            memcpy(st[j], buf, sizeof(i32) * (size_t)len);
            stlen[j] = len;
            next[j] = head[mn];
            head[mn] = j;
        }
    }
    for (i32 j = 0; j < n; j++) free(st[j]);
    free(iperm); free(mark); free(st); free(stlen); free(head); free(next); free(buf);
    return ORC_OK;
}

/* Postorder of a forest: roots in ascending id, children in ascending id,
 * every node right after its children.  post[k] = node placed at k. */
int orc_postorder(i32 n, const i32* parent, i32* post)
{
    i32* head = (i32*)malloc(sizeof(i32) * ((size_t)n + 1));
    i32* next = (i32*)malloc(sizeof(i32) * ((size_t)n + 1));
    i32* stack = (i32*)malloc(sizeof(i32) * ((size_t)n + 1));
    i32* it = (i32*)malloc(sizeof(i32) * ((size_t)n + 1));
    if (!head || !next || !stack || !it) return ORC_ENOMEM;
    for (i32 v = 0; v < n; v++) head[v] = -1;
    /* children lists in ascending order: insert in descending order at the front */
    for (i32 v = n - 1; v >= 0; v--)
        if (parent[v] >= 0) { next[v] = head[parent[v]]; head[parent[v]] = v; }
    i32 k = 0;
    for (i32 r = 0; r < n; r++) {
        if (parent[r] >= 0) continue;
        i32 top = 0;
        stack[top] = r; it[top] = head[r];
        while (top >= 0) {
            if (it[top] >= 0) {
                i32 ch = it[top];
                it[top] = next[ch];
                top++;
                stack[top] = ch; it[top] = head[ch];
            } else {
                post[k++] = stack[top];
                top--;
            }
        }
    }
    free(head); free(next); free(stack); free(it);
    return k == n ? ORC_OK : ORC_EINVAL;
}

/* ------------------------------------------------------------------ */
/* Binary min-heap keyed (cost, id), for the amalgamation.               */
/* ------------------------------------------------------------------ */
typedef struct { i64 cost; i32 id; } hent;
typedef struct { hent* a; i64 n, cap; } heap_t;

static int hless(hent x, hent y) { return x.cost < y.cost || (x.cost == y.cost && x.id < y.id); }

static void hpush(heap_t* h, i64 cost, i32 id)
{
    if (h->n == h->cap) { h->cap = h->cap ? 2 * h->cap : 1024; h->a = (hent*)realloc(h->a, sizeof(hent) * (size_t)h->cap); }
    i64 i = h->n++;
    hent e; e.cost = cost; e.id = id;
    while (i > 0) {
        i64 p = (i - 1) / 2;
        if (!hless(e, h->a[p])) break;
        h->a[i] = h->a[p];
        i = p;
    }
    h->a[i] = e;
}

static hent hpop(heap_t* h)
{
    hent top = h->a[0];
    hent last = h->a[--h->n];
    i64 i = 0;
    for (;;) {
        i64 l = 2 * i + 1, r = l + 1, s = i;
        hent best = last;
        if (l < h->n && hless(h->a[l], best)) { s = l; best = h->a[l]; }
        if (r < h->n && hless(h->a[r], best)) { s = r; }
        if (s == i) break;
        h->a[i] = h->a[s];
        i = s;
    }
    if (h->n > 0) h->a[i] = last;
    return top;
}

/* ------------------------------------------------------------------ */
/* The symbolic result (exported arrays).                                */
/* ------------------------------------------------------------------ */
typedef struct {
    i32 n;
    i32* perm;   /* new -> old */
    i32* iperm;  /* old -> new */
    i32* etree;  /* column elimination tree in the final numbering */
    i32 nsn_fund, nsn;
    i32* snptr;  /* [nsn+1] first column of every amalgamated supernode */
    i32 ncblk;
    i32* fcol; i32* lcol; i32* stride; i64* panel_off; i32* bptr; i32* cparent;
    i32 nblok;
    i32* frow; i32* lrow; i32* fcblk; i32* coefind;
    i32* uptr; i32* utgt; i32* dep;
    i64 nupd;
    i64 nnz_exact, nnz_amalg, zeros_used, budget, panel_size;
    double flops_alg, flops_exec;
    double flops_alg_lu, flops_exec_lu;   /* L U count (Section IV's flop totals; our formula) */
    i64* colcount; /* exact column counts (diagonal included), final numbering */
} orc_sym;

void orc_free(orc_sym* s)
{
    if (!s) return;
    free(s->perm); free(s->iperm); free(s->etree); free(s->snptr);
    free(s->fcol); free(s->lcol); free(s->stride); free(s->panel_off); free(s->bptr); free(s->cparent);
    free(s->frow); free(s->lrow); free(s->fcblk); free(s->coefind);
    free(s->uptr); free(s->utgt); free(s->dep); free(s->colcount);
    free(s);
}

/*
 * Full analysis.  Steps (each reading documented at its function):
 *   O1 graph, O2 nested dissection (or the user's permutation), O3 etree +
 *   postorder, O4 column counts and fundamental supernodes, O5 amalgamation
 *   with a fill budget of amalg_pct percent (the paper allows up to 12%),
 *   O6 final postorder, O7 vertical split of supernodes wider than
 *   split_width, O8 blocks (maximal runs of consecutive rows facing one
 *   column block), update pairs and dependency counts, O9 flop counts.
 */
int orc_analyze(i32 n, const i64* colptr, const i32* rowind, i32 leaf, i32 amalg_pct, i32 split_width,
                const i32* user_perm, orc_sym** out)
{
    if (n < 0 || split_width < 1 || amalg_pct < 0) return ORC_EINVAL;
    for (i32 j = 0; j < n; j++) {
        if (colptr[j + 1] < colptr[j]) return ORC_EINVAL;
        for (i64 p = colptr[j]; p < colptr[j + 1]; p++) {
            if (rowind[p] < 0 || rowind[p] >= n) return ORC_EINVAL;
            if (p > colptr[j] && rowind[p] <= rowind[p - 1]) return ORC_EINVAL;
        }
    }
    orc_sym* s = (orc_sym*)calloc(1, sizeof(orc_sym));
    s->n = n;
    i64 nnz = colptr[n];
    i64* xadj = (i64*)malloc(sizeof(i64) * ((size_t)n + 1));
    i32* adj = (i32*)malloc(sizeof(i32) * ((size_t)2 * (size_t)nnz + 1));
    orc_graph(n, colptr, rowind, xadj, adj);

    /* O2 */
    i32* p0 = (i32*)malloc(sizeof(i32) * ((size_t)n + 1));
    if (user_perm) {
        char* seenv = (char*)calloc((size_t)n + 1, 1);
        for (i32 k = 0; k < n; k++) {
            if (user_perm[k] < 0 || user_perm[k] >= n || seenv[user_perm[k]]) { free(seenv); return ORC_EINVAL; }
            seenv[user_perm[k]] = 1;
            p0[k] = user_perm[k];
        }
        free(seenv);
    } else {
        orc_nd(n, xadj, adj, leaf, p0);
    }

    /* O3: etree of the ND ordering, postorder, relabel */
    i32* par0 = (i32*)malloc(sizeof(i32) * ((size_t)n + 1));
    i64* eta0 = (i64*)malloc(sizeof(i64) * ((size_t)n + 1));
    orc_etree_counts(n, xadj, adj, p0, par0, eta0);
    i32* post = (i32*)malloc(sizeof(i32) * ((size_t)n + 1));
    orc_postorder(n, par0, post);
    i32* ipost = (i32*)malloc(sizeof(i32) * ((size_t)n + 1));
    for (i32 k = 0; k < n; k++) ipost[post[k]] = k;
    i32* p1 = (i32*)malloc(sizeof(i32) * ((size_t)n + 1));   /* O3 label -> original */
    i32* par1 = (i32*)malloc(sizeof(i32) * ((size_t)n + 1));
    i64* eta = (i64*)malloc(sizeof(i64) * ((size_t)n + 1));
    for (i32 k = 0; k < n; k++) {
        p1[k] = p0[post[k]];
        par1[k] = par0[post[k]] < 0 ? -1 : ipost[par0[post[k]]];
        eta[k] = eta0[post[k]];
    }
    i32* ip1 = (i32*)malloc(sizeof(i32) * ((size_t)n + 1));
    for (i32 k = 0; k < n; k++) ip1[p1[k]] = k;

    /* O4: fundamental supernodes */
    i32* nchild = (i32*)calloc((size_t)n + 1, sizeof(i32));
    for (i32 j = 0; j < n; j++) if (par1[j] >= 0) nchild[par1[j]]++;
    i32* fsn_of = (i32*)malloc(sizeof(i32) * ((size_t)n + 1));
    i32* fstart = (i32*)malloc(sizeof(i32) * ((size_t)n + 2));
    i32 nf = 0;
    for (i32 j = 0; j < n; j++) {
        int join = j > 0 && par1[j - 1] == j && nchild[j] == 1 && eta[j - 1] == eta[j] + 1;
        if (!join) fstart[nf++] = j;
        fsn_of[j] = nf - 1;
    }
    fstart[nf] = n;
    s->nsn_fund = nf;
    i64 nnz_exact = 0;
    double flops_alg = 0.0;
    double flops_alg_lu = 0.0;
    for (i32 j = 0; j < n; j++) {
        nnz_exact += eta[j];
        flops_alg += (double)eta[j] * (double)eta[j];
        flops_alg_lu += 2.0 * (double)(eta[j] - 1) * (double)(eta[j] - 1) + (double)(eta[j] - 1);
    }

    /* R_s for fundamental supernodes: supernodal merge over children (O3 labels). */
    i32* fw = (i32*)malloc(sizeof(i32) * ((size_t)nf + 1));
    i32* fpar = (i32*)malloc(sizeof(i32) * ((size_t)nf + 1));
    i32** R = (i32**)calloc((size_t)nf + 1, sizeof(i32*));
    i32* rlen = (i32*)calloc((size_t)nf + 1, sizeof(i32));
    i32* chead = (i32*)malloc(sizeof(i32) * ((size_t)nf + 1));
    i32* cnext = (i32*)malloc(sizeof(i32) * ((size_t)nf + 1));
    i32* mark = (i32*)malloc(sizeof(i32) * ((size_t)n + 1));
    i32* buf = (i32*)malloc(sizeof(i32) * ((size_t)n + 1));
    for (i32 j = 0; j < n; j++) mark[j] = -1;
    for (i32 f = 0; f < nf; f++) {
        fw[f] = fstart[f + 1] - fstart[f];
        i32 last = fstart[f + 1] - 1;
        fpar[f] = par1[last] < 0 ? -1 : fsn_of[par1[last]];
        chead[f] = -1;
    }
    for (i32 f = nf - 1; f >= 0; f--)
        if (fpar[f] >= 0) { cnext[f] = chead[fpar[f]]; chead[fpar[f]] = f; }
    for (i32 f = 0; f < nf; f++) {
        i32 last = fstart[f + 1] - 1, len = 0;
        for (i32 j = fstart[f]; j <= last; j++) {
            i32 oj = p1[j];
            for (i64 p = xadj[oj]; p < xadj[oj + 1]; p++) {
                i32 i = ip1[adj[p]];
                if (i > last && mark[i] != f) { mark[i] = f; buf[len++] = i; }
            }
        }
        for (i32 c = chead[f]; c >= 0; c = cnext[c])
            for (i32 q = 0; q < rlen[c]; q++) {
                i32 i = R[c][q];
                if (i > last && mark[i] != f) { mark[i] = f; buf[len++] = i; }
            }
        qsort(buf, (size_t)len, sizeof(i32), cmp_i32);
        R[f] = (i32*)malloc(sizeof(i32) * ((size_t)len + 1));
        memcpy(R[f], buf, sizeof(i32) * (size_t)len);
        rlen[f] = len;
        if ((i64)len != eta[last] - 1) { /* symbolic inconsistency */
            return ORC_EINVAL;
        }
    }

    /* O5: amalgamation, greedy by (cost, id) with an integer fill budget. */
    i64 budget = ((i64)amalg_pct * nnz_exact) / 100;
    i64* cost = (i64*)calloc((size_t)nf + 1, sizeof(i64));
    char* alive = (char*)malloc((size_t)nf + 1);
    i32* w = (i32*)malloc(sizeof(i32) * ((size_t)nf + 1));
    i32* spar = (i32*)malloc(sizeof(i32) * ((size_t)nf + 1));
    i32* mhead = (i32*)malloc(sizeof(i32) * ((size_t)nf + 1)); /* member lists */
    i32* mtail = (i32*)malloc(sizeof(i32) * ((size_t)nf + 1));
    i32* mnext = (i32*)malloc(sizeof(i32) * ((size_t)nf + 1));
    heap_t hp; memset(&hp, 0, sizeof(hp));
    for (i32 f = 0; f < nf; f++) {
        alive[f] = 1; w[f] = fw[f]; spar[f] = fpar[f];
        mhead[f] = f; mtail[f] = f; mnext[f] = -1;
    }
    for (i32 f = 0; f < nf; f++)
        if (spar[f] >= 0) {
            i32 p = spar[f];
            cost[f] = (i64)w[f] * ((i64)w[p] + rlen[p] - rlen[f]);
            hpush(&hp, cost[f], f);
        }
    i64 used = 0;
    while (hp.n > 0) {
        hent e = hpop(&hp);
        i32 c = e.id;
        if (!alive[c] || spar[c] < 0 || e.cost != cost[c]) continue;
        if (used + e.cost > budget) break;
        i32 p = spar[c];
        used += e.cost;
        w[p] += w[c];
        alive[c] = 0;
        mnext[mtail[p]] = mhead[c]; /* member list: order does not matter, columns are sorted later */
        mtail[p] = mtail[c];
        /* remove c from p's children */
        i32* link = &chead[p];
        while (*link != c) link = &cnext[*link];
        *link = cnext[c];
        /* adopt c's children */
        for (i32 x = chead[c]; x >= 0;) {
            i32 nx = cnext[x];
            spar[x] = p;
            cnext[x] = chead[p];
            chead[p] = x;
            x = nx;
        }
        chead[c] = -1;
        if (spar[p] >= 0) {
            i32 q = spar[p];
            cost[p] = (i64)w[p] * ((i64)w[q] + rlen[q] - rlen[p]);
            hpush(&hp, cost[p], p);
        }
        for (i32 x = chead[p]; x >= 0; x = cnext[x]) {
            cost[x] = (i64)w[x] * ((i64)w[p] + rlen[p] - rlen[x]);
            hpush(&hp, cost[x], x);
        }
    }
    free(hp.a);
    s->zeros_used = used;
    s->budget = budget;
    s->nnz_exact = nnz_exact;
    s->nnz_amalg = nnz_exact + used;
    s->flops_alg = flops_alg;
    s->flops_alg_lu = flops_alg_lu;

    /* O6: postorder of the amalgamated tree (ids = surviving fundamental index). */
    i32* apar = (i32*)malloc(sizeof(i32) * ((size_t)nf + 1));
    for (i32 f = 0; f < nf; f++) apar[f] = alive[f] ? spar[f] : -2;
    /* compact live nodes, keep ascending id */
    i32* live = (i32*)malloc(sizeof(i32) * ((size_t)nf + 1));
    i32* lid = (i32*)malloc(sizeof(i32) * ((size_t)nf + 1));
    i32 nsn = 0;
    for (i32 f = 0; f < nf; f++) if (alive[f]) { lid[f] = nsn; live[nsn++] = f; }
    i32* cpar = (i32*)malloc(sizeof(i32) * ((size_t)nsn + 1));
    for (i32 a = 0; a < nsn; a++) cpar[a] = apar[live[a]] < 0 ? -1 : lid[apar[live[a]]];
    i32* apost = (i32*)malloc(sizeof(i32) * ((size_t)nsn + 1));
    orc_postorder(nsn, cpar, apost);
    s->nsn = nsn;
    s->snptr = (i32*)malloc(sizeof(i32) * ((size_t)nsn + 1));
    s->perm = (i32*)malloc(sizeof(i32) * ((size_t)n + 1));
    s->iperm = (i32*)malloc(sizeof(i32) * ((size_t)n + 1));
    i32* lab3to4 = (i32*)malloc(sizeof(i32) * ((size_t)n + 1)); /* O3 label -> final */
    i32* snR = (i32*)malloc(sizeof(i32) * ((size_t)nsn + 1)); /* fundamental id holding R of the node */
    i32 col = 0;
    for (i32 t = 0; t < nsn; t++) {
        i32 f = live[apost[t]];
        s->snptr[t] = col;
        i32 cnt = 0;
        for (i32 m = mhead[f]; m >= 0; m = mnext[m])
            for (i32 j = fstart[m]; j < fstart[m + 1]; j++) buf[cnt++] = j;
        qsort(buf, (size_t)cnt, sizeof(i32), cmp_i32);
        for (i32 q = 0; q < cnt; q++) { lab3to4[buf[q]] = col; s->perm[col] = p1[buf[q]]; col++; }
        snR[t] = f;
    }
    s->snptr[nsn] = col;
    for (i32 k = 0; k < n; k++) s->iperm[s->perm[k]] = k;
    s->etree = (i32*)malloc(sizeof(i32) * ((size_t)n + 1));
    s->colcount = (i64*)malloc(sizeof(i64) * ((size_t)n + 1));
    for (i32 j = 0; j < n; j++) s->colcount[lab3to4[j]] = eta[j];
    for (i32 j = 0; j < n; j++) {
        i32 pj = par1[j];
        s->etree[lab3to4[j]] = pj < 0 ? -1 : lab3to4[pj];
    }

    /* O7: vertical split; O8: blocks. */
    i32 ncblk = 0;
    for (i32 t = 0; t < nsn; t++) {
        i32 wd = s->snptr[t + 1] - s->snptr[t];
        ncblk += (wd + split_width - 1) / split_width;
    }
    s->ncblk = ncblk;
    s->fcol = (i32*)malloc(sizeof(i32) * ((size_t)ncblk + 1));
    s->lcol = (i32*)malloc(sizeof(i32) * ((size_t)ncblk + 1));
    i32* csn = (i32*)malloc(sizeof(i32) * ((size_t)ncblk + 1));
    i32 kk = 0;
    double flops_exec = 0.0, flops_exec_lu = 0.0;
    for (i32 t = 0; t < nsn; t++) {
        i32 f0 = s->snptr[t], wd = s->snptr[t + 1] - f0;
        i32 np = (wd + split_width - 1) / split_width;
        i32 base = wd / np, extra = wd % np, c0 = f0;
        for (i32 q = 0; q < np; q++) {
            i32 ww = base + (q < extra ? 1 : 0);
            s->fcol[kk] = c0; s->lcol[kk] = c0 + ww - 1; csn[kk] = t; kk++;
            c0 += ww;
        }
        i32 rl = rlen[snR[t]];
        for (i32 i = 0; i < wd; i++) {
            double e2 = (double)(wd - i + rl);
            flops_exec += e2 * e2;
            flops_exec_lu += 2.0 * (e2 - 1.0) * (e2 - 1.0) + (e2 - 1.0);
        }
    }
    s->flops_exec = flops_exec;
    s->flops_exec_lu = flops_exec_lu;
    i32* col2cblk = (i32*)malloc(sizeof(i32) * ((size_t)n + 1));
    for (i32 k = 0; k < ncblk; k++) for (i32 j = s->fcol[k]; j <= s->lcol[k]; j++) col2cblk[j] = k;

    /* count blocks */
    i32 nblok = 0;
    i32* rows = buf;
    for (int pass = 0; pass < 2; pass++) {
        i32 b = 0;
        i64 off = 0;
        for (i32 k = 0; k < ncblk; k++) {
            i32 t = csn[k];
            i32 ln = 0;
            for (i32 j = s->lcol[k] + 1; j < s->snptr[t + 1]; j++) rows[ln++] = j;
            i32 f = snR[t];
            i32 rstart = ln;
            for (i32 q = 0; q < rlen[f]; q++) rows[ln++] = lab3to4[R[f][q]];
            qsort(rows + rstart, (size_t)(ln - rstart), sizeof(i32), cmp_i32);
            i32 wd = s->lcol[k] - s->fcol[k] + 1;
            if (pass == 1) {
                s->bptr[k] = b;
                s->frow[b] = s->fcol[k]; s->lrow[b] = s->lcol[k]; s->fcblk[b] = k; s->coefind[b] = 0;
            }
            b++;
            i32 h = wd;
            for (i32 q = 0; q < ln;) {
                i32 q2 = q;
                while (q2 + 1 < ln && rows[q2 + 1] == rows[q2] + 1 && col2cblk[rows[q2 + 1]] == col2cblk[rows[q]]) q2++;
                if (pass == 1) {
                    s->frow[b] = rows[q]; s->lrow[b] = rows[q2]; s->fcblk[b] = col2cblk[rows[q]]; s->coefind[b] = h;
                }
                h += q2 - q + 1;
                b++;
                q = q2 + 1;
            }
            if (pass == 1) { s->stride[k] = h; s->panel_off[k] = off; }
            off += (i64)h * wd;
        }
        if (pass == 0) {
            nblok = b;
            s->nblok = nblok;
            s->bptr = (i32*)malloc(sizeof(i32) * ((size_t)ncblk + 1));
            s->frow = (i32*)malloc(sizeof(i32) * ((size_t)nblok + 1));
            s->lrow = (i32*)malloc(sizeof(i32) * ((size_t)nblok + 1));
            s->fcblk = (i32*)malloc(sizeof(i32) * ((size_t)nblok + 1));
            s->coefind = (i32*)malloc(sizeof(i32) * ((size_t)nblok + 1));
            s->stride = (i32*)malloc(sizeof(i32) * ((size_t)ncblk + 1));
            s->panel_off = (i64*)malloc(sizeof(i64) * ((size_t)ncblk + 1));
        } else {
            s->bptr[ncblk] = b;
            s->panel_off[ncblk] = off;
            s->panel_size = off;
        }
    }
    /* update pairs, dependency counts, cblk parent */
    s->uptr = (i32*)malloc(sizeof(i32) * ((size_t)ncblk + 1));
    s->dep = (i32*)calloc((size_t)ncblk + 1, sizeof(i32));
    s->cparent = (i32*)malloc(sizeof(i32) * ((size_t)ncblk + 1));
    i64 nup = 0;
    for (i32 k = 0; k < ncblk; k++) {
        i32 prev = -1;
        for (i32 b = s->bptr[k] + 1; b < s->bptr[k + 1]; b++)
            if (s->fcblk[b] != prev) { prev = s->fcblk[b]; nup++; }
    }
    s->utgt = (i32*)malloc(sizeof(i32) * ((size_t)nup + 1));
    s->nupd = nup;
    nup = 0;
    for (i32 k = 0; k < ncblk; k++) {
        s->uptr[k] = (i32)nup;
        i32 prev = -1;
        s->cparent[k] = s->bptr[k + 1] > s->bptr[k] + 1 ? s->fcblk[s->bptr[k] + 1] : -1;
        for (i32 b = s->bptr[k] + 1; b < s->bptr[k + 1]; b++)
            if (s->fcblk[b] != prev) { prev = s->fcblk[b]; s->utgt[nup++] = prev; s->dep[prev]++; }
    }
    s->uptr[ncblk] = (i32)nup;

    for (i32 f = 0; f < nf; f++) free(R[f]);
    free(R); free(rlen); free(xadj); free(adj); free(p0); free(par0); free(eta0); free(post); free(ipost);
    free(p1); free(par1); free(eta); free(ip1); free(nchild); free(fsn_of); free(fstart); free(fw); free(fpar);
    free(chead); free(cnext); free(mark); free(buf); free(cost); free(alive); free(w); free(spar);
    free(mhead); free(mtail); free(mnext); free(apar); free(live); free(lid); free(cpar); free(apost);
    free(lab3to4); free(snR); free(csn); free(col2cblk);
    *out = s;
    return ORC_OK;
}

/* Accessors for the Python driver. */
i32 orc_sym_int(const orc_sym* s, int what)
{
    switch (what) {
    case 0: return s->n;
    case 1: return s->ncblk;
    case 2: return s->nblok;
    case 3: return s->nsn;
    case 4: return s->nsn_fund;
    case 5: return (i32)s->nupd;
    default: return -1;
    }
}

i64 orc_sym_i64(const orc_sym* s, int what)
{
    switch (what) {
    case 0: return s->nnz_exact;
    case 1: return s->nnz_amalg;
    case 2: return s->zeros_used;
    case 3: return s->budget;
    case 4: return s->panel_size;
    default: return -1;
    }
}

double orc_sym_dbl(const orc_sym* s, int what)
{
    return what == 0 ? s->flops_alg : what == 1 ? s->flops_exec : what == 2 ? s->flops_alg_lu : s->flops_exec_lu;
}

/* Copy one exported array out; names are numbered (see the Python driver). */
int orc_sym_copy(const orc_sym* s, int what, void* dst)
{
    size_t n = (size_t)s->n, nc = (size_t)s->ncblk, nb = (size_t)s->nblok;
    switch (what) {
    case 0: memcpy(dst, s->perm, 4 * n); break;
    case 1: memcpy(dst, s->iperm, 4 * n); break;
    case 2: memcpy(dst, s->etree, 4 * n); break;
    case 3: memcpy(dst, s->snptr, 4 * ((size_t)s->nsn + 1)); break;
    case 4: memcpy(dst, s->fcol, 4 * nc); break;
    case 5: memcpy(dst, s->lcol, 4 * nc); break;
    case 6: memcpy(dst, s->stride, 4 * nc); break;
    case 7: memcpy(dst, s->panel_off, 8 * (nc + 1)); break;
    case 8: memcpy(dst, s->bptr, 4 * (nc + 1)); break;
    case 9: memcpy(dst, s->cparent, 4 * nc); break;
    case 10: memcpy(dst, s->frow, 4 * nb); break;
    case 11: memcpy(dst, s->lrow, 4 * nb); break;
    case 12: memcpy(dst, s->fcblk, 4 * nb); break;
    case 13: memcpy(dst, s->coefind, 4 * nb); break;
    case 14: memcpy(dst, s->uptr, 4 * (nc + 1)); break;
    case 15: memcpy(dst, s->utgt, 4 * (size_t)s->nupd); break;
    case 16: memcpy(dst, s->dep, 4 * nc); break;
    case 17: memcpy(dst, s->colcount, 8 * n); break;
    default: return ORC_EINVAL;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Numeric part.                                                        */
/* ------------------------------------------------------------------ */

/* Panel row index -> position inside cblk k of global row r (r in its structure). */
static i32 row_pos(const orc_sym* s, i32 k, i32 r)
{
    if (r >= s->fcol[k] && r <= s->lcol[k]) return r - s->fcol[k];
    for (i32 b = s->bptr[k] + 1; b < s->bptr[k + 1]; b++)
        if (r >= s->frow[b] && r <= s->lrow[b]) return s->coefind[b] + (r - s->frow[b]);
    return -1;
}

/*
 * Assembly: zero the panels, then add every entry of the lower triangle of A
 * (original row >= original column) at its place in P A P^T's lower
 * triangle.  Panels are column-major, leading dimension = stride[k].
 */
int orc_assemble(const orc_sym* s, const i64* colptr, const i32* rowind, const double* val, double* P)
{
    memset(P, 0, sizeof(double) * (size_t)s->panel_size);
    i32* col2cblk = (i32*)malloc(sizeof(i32) * ((size_t)s->n + 1));
    for (i32 k = 0; k < s->ncblk; k++) for (i32 j = s->fcol[k]; j <= s->lcol[k]; j++) col2cblk[j] = k;
    for (i32 j = 0; j < s->n; j++)
        for (i64 p = colptr[j]; p < colptr[j + 1]; p++) {
            i32 i = rowind[p];
            if (i < j) continue;
            i32 a = s->iperm[i], b = s->iperm[j];
            i32 r = a > b ? a : b, c = a > b ? b : a;
            i32 k = col2cblk[c];
            i32 pos = row_pos(s, k, r);
            if (pos < 0) { free(col2cblk); return ORC_EINVAL; }
            P[s->panel_off[k] + (i64)(c - s->fcol[k]) * s->stride[k] + pos] += val[p];
        }
    free(col2cblk);
    return ORC_OK;
}

/*
 * The same assembly for the column blocks k0..k1-1 only: their panels are
 * zeroed and receive the entries whose (permuted) column they hold; other
 * panels are left as they are.  Used to time the factorization of one
 * subtree of the block elimination tree without assembling the whole matrix.
 */
int orc_assemble_range(const orc_sym* s, const i64* colptr, const i32* rowind, const double* val, double* P,
                       i32 k0, i32 k1)
{
    if (k0 < 0) k0 = 0;
    if (k1 > s->ncblk) k1 = s->ncblk;
    if (k0 >= k1) return ORC_OK;
    memset(P + s->panel_off[k0], 0, sizeof(double) * (size_t)(s->panel_off[k1] - s->panel_off[k0]));
    const i32 c0 = s->fcol[k0], c1 = s->lcol[k1 - 1];
    i32* col2cblk = (i32*)malloc(sizeof(i32) * ((size_t)s->n + 1));
    if (!col2cblk) return ORC_ENOMEM;
    for (i32 k = 0; k < s->ncblk; k++) for (i32 j = s->fcol[k]; j <= s->lcol[k]; j++) col2cblk[j] = k;
    for (i32 j = 0; j < s->n; j++)
        for (i64 p = colptr[j]; p < colptr[j + 1]; p++) {
            i32 i = rowind[p];
            if (i < j) continue;
            i32 a = s->iperm[i], b = s->iperm[j];
            i32 r = a > b ? a : b, c = a > b ? b : a;
            if (c < c0 || c > c1) continue;
            i32 k = col2cblk[c];
            i32 pos = row_pos(s, k, r);
            if (pos < 0) { free(col2cblk); return ORC_EINVAL; }
            P[s->panel_off[k] + (i64)(c - s->fcol[k]) * s->stride[k] + pos] += val[p];
        }
    free(col2cblk);
    return ORC_OK;
}

/*
 * Right-looking supernodal LL^T in ascending column-block order
 * (Section III, steps 1-3 of the 1D task; Section V-B CPU update scheme):
 *   1. Cholesky of the diagonal block, column by column; breakdown when a
 *      pivot is not > 0 (NaN included);
 *   2. the off-diagonal rows are solved against L_kk^T row by row;
 *   3. for every facing column block j (ascending), the outer product of
 *      the rows from the first block facing j to the end of the panel with
 *      the facing rows is formed in a temporary buffer (inner index
 *      ascending) and subtracted at its place in panel j; only the lower
 *      triangle of j's diagonal block is touched.
 * Returns ORC_ENOTPD and the failing column (final numbering) on breakdown.
 */
int orc_factor_range(const orc_sym* s, double* P, i32 kbeg, i32 kend, i32* fail_col);

int orc_factor(const orc_sym* s, double* P, i32* fail_col) { return orc_factor_range(s, P, 0, s->ncblk, fail_col); }

/* Column blocks 0..kend-1 only: after it they hold their final values (every
 * update into them comes from a smaller block). */
int orc_factor_upto(const orc_sym* s, double* P, i32 kend, i32* fail_col)
{
    return orc_factor_range(s, P, 0, kend, fail_col);
}

/* Column blocks kbeg..kend-1 only (their updates into later blocks
 * included).  When kbeg..kend-1 is a whole subtree of the block elimination
 * tree (the descendants of kend-1 and itself, consecutive in the postorder),
 * every update into these blocks comes from inside the range, so they hold
 * their final values afterwards. */
int orc_factor_range(const orc_sym* s, double* P, i32 kbeg, i32 kend, i32* fail_col)
{
    *fail_col = -1;
    if (kend > s->ncblk) kend = s->ncblk;
    if (kbeg < 0) kbeg = 0;
    i32 maxs = 0;
    for (i32 k = 0; k < s->ncblk; k++) if (s->stride[k] > maxs) maxs = s->stride[k];
    double* W = (double*)malloc(sizeof(double) * (size_t)maxs * (size_t)maxs + 8);
    i32* grow = (i32*)malloc(sizeof(i32) * ((size_t)maxs + 1));
    if (!W || !grow) return ORC_ENOMEM;
    for (i32 k = kbeg; k < kend; k++) {
        i32 wd = s->lcol[k] - s->fcol[k] + 1, ld = s->stride[k];
        double* L = P + s->panel_off[k];
        /* global row of each panel row */
        for (i32 b = s->bptr[k]; b < s->bptr[k + 1]; b++)
            for (i32 r = s->frow[b]; r <= s->lrow[b]; r++) grow[s->coefind[b] + r - s->frow[b]] = r;
        /* 1. diagonal block */
        for (i32 c = 0; c < wd; c++) {
            double d = L[c + (i64)c * ld];
            for (i32 p = 0; p < c; p++) d -= L[c + (i64)p * ld] * L[c + (i64)p * ld];
            if (!(d > 0.0)) { *fail_col = s->fcol[k] + c; free(W); free(grow); return ORC_ENOTPD; }
            d = sqrt(d);
            L[c + (i64)c * ld] = d;
            for (i32 r = c + 1; r < wd; r++) {
                double v = L[r + (i64)c * ld];
                for (i32 p = 0; p < c; p++) v -= L[r + (i64)p * ld] * L[c + (i64)p * ld];
                L[r + (i64)c * ld] = v / d;
            }
        }
        /* 2. triangular solve of the off-diagonal rows */
        for (i32 r = wd; r < ld; r++)
            for (i32 c = 0; c < wd; c++) {
                double v = L[r + (i64)c * ld];
                for (i32 p = 0; p < c; p++) v -= L[r + (i64)p * ld] * L[c + (i64)p * ld];
                L[r + (i64)c * ld] = v / L[c + (i64)c * ld];
            }
        /* 3. updates of the facing panels */
        for (i32 b = s->bptr[k] + 1; b < s->bptr[k + 1];) {
            i32 j = s->fcblk[b];
            i32 b2 = b;
            while (b2 < s->bptr[k + 1] && s->fcblk[b2] == j) b2++;
            i32 rs = s->coefind[b];
            i32 nf = s->coefind[b2 - 1] + (s->lrow[b2 - 1] - s->frow[b2 - 1] + 1) - rs;
            i32 m = ld - rs;
            for (i32 q = 0; q < nf; q++)
                for (i32 i = 0; i < m; i++) {
                    double acc = 0.0;
                    for (i32 p = 0; p < wd; p++) acc += L[rs + i + (i64)p * ld] * L[rs + q + (i64)p * ld];
                    W[i + (i64)q * m] = acc;
                }
            double* T = P + s->panel_off[j];
            i32 ldj = s->stride[j];
            for (i32 q = 0; q < nf; q++) {
                i32 gc = grow[rs + q];
                i32 tc = gc - s->fcol[j];
                for (i32 i = 0; i < m; i++) {
                    i32 gr = grow[rs + i];
                    if (gr < gc) continue;
                    i32 pos = row_pos(s, j, gr);
                    if (pos < 0) { free(W); free(grow); return ORC_EINVAL; }
                    T[(i64)tc * ldj + pos] -= W[i + (i64)q * m];
                }
            }
            b = b2;
        }
    }
    free(W);
    free(grow);
    return ORC_OK;
}

/*
 * Right-looking supernodal L D L^T, the variant of the same method that
 * Section III names (no dynamic pivoting: the elimination order is the
 * analysis' order).  Same steps and order as the LL^T factorization above,
 * with D applied inside each update product (one of the two update forms
 * Section V compares):
 *   1. L D L^T of the diagonal block, column by column:
 *        d_c  = a_cc - sum_{p<c} l_cp d_p l_cp,
 *        l_rc = (a_rc - sum_{p<c} l_rp d_p l_cp) / d_c   (r > c);
 *      breakdown when a pivot is zero or not finite;
 *   2. the off-diagonal rows by the same formula for l_rc;
 *   3. every facing panel j gets W = L_rows D L_facing^T subtracted.
 * Storage: D on the diagonal of each diagonal block, the strictly lower
 * entries of L (unit diagonal implied) below it and in the off-diagonal
 * rows.  Returns ORC_ENOTPD and the failing column on breakdown.
 */
int orc_factor_ldlt_sp(const orc_sym* s, double* P, double tau, i32* nrep, i32* fail_col);

int orc_factor_ldlt(const orc_sym* s, double* P, i32* fail_col)
{
    i32 nrep = 0;
    return orc_factor_ldlt_sp(s, P, 0.0, &nrep, fail_col);
}

/*
 * Static pivot replacement (Section III's static pivoting: no row or column
 * exchange, so a pivot that is too small is replaced instead): with
 * tau > 0, a pivot of magnitude below tau becomes +tau or -tau with the
 * pivot's sign (+tau for a zero pivot), and *nrep counts the replacements;
 * tau = 0 leaves every pivot as it is (a zero or non-finite one is then a
 * breakdown).  A non-finite pivot is never replaced.
 */
static double static_pivot(double d, double tau, i32* nrep)
{
    if (tau > 0.0 && fabs(d) < tau) {
        (*nrep)++;
        return d < 0.0 ? -tau : tau;
    }
    return d;
}

int orc_factor_ldlt_sp(const orc_sym* s, double* P, double tau, i32* nrep, i32* fail_col)
{
    *fail_col = -1;
    *nrep = 0;
    i32 maxs = 0;
    for (i32 k = 0; k < s->ncblk; k++) if (s->stride[k] > maxs) maxs = s->stride[k];
    double* W = (double*)malloc(sizeof(double) * (size_t)maxs * (size_t)maxs + 8);
    i32* grow = (i32*)malloc(sizeof(i32) * ((size_t)maxs + 1));
    if (!W || !grow) return ORC_ENOMEM;
    for (i32 k = 0; k < s->ncblk; k++) {
        i32 wd = s->lcol[k] - s->fcol[k] + 1, ld = s->stride[k];
        double* L = P + s->panel_off[k];
        for (i32 b = s->bptr[k]; b < s->bptr[k + 1]; b++)
            for (i32 r = s->frow[b]; r <= s->lrow[b]; r++) grow[s->coefind[b] + r - s->frow[b]] = r;
        /* 1. diagonal block; 2. the rows below use the same formula */
        for (i32 c = 0; c < wd; c++) {
            double d = L[c + (i64)c * ld];
            for (i32 p = 0; p < c; p++) d -= L[c + (i64)p * ld] * L[p + (i64)p * ld] * L[c + (i64)p * ld];
            d = static_pivot(d, tau, nrep);
            if (!(d != 0.0) || !isfinite(d)) { *fail_col = s->fcol[k] + c; free(W); free(grow); return ORC_ENOTPD; }
            L[c + (i64)c * ld] = d;
            for (i32 r = c + 1; r < ld; r++) {
                double v = L[r + (i64)c * ld];
                for (i32 p = 0; p < c; p++) v -= L[r + (i64)p * ld] * L[p + (i64)p * ld] * L[c + (i64)p * ld];
                L[r + (i64)c * ld] = v / d;
            }
        }
        /* 3. updates of the facing panels: W = L_rows D L_facing^T */
        for (i32 b = s->bptr[k] + 1; b < s->bptr[k + 1];) {
            i32 j = s->fcblk[b];
            i32 b2 = b;
            while (b2 < s->bptr[k + 1] && s->fcblk[b2] == j) b2++;
            i32 rs = s->coefind[b];
            i32 nf = s->coefind[b2 - 1] + (s->lrow[b2 - 1] - s->frow[b2 - 1] + 1) - rs;
            i32 m = ld - rs;
            for (i32 q = 0; q < nf; q++)
                for (i32 i = 0; i < m; i++) {
                    double acc = 0.0;
                    for (i32 p = 0; p < wd; p++)
                        acc += L[rs + i + (i64)p * ld] * L[p + (i64)p * ld] * L[rs + q + (i64)p * ld];
                    W[i + (i64)q * m] = acc;
                }
            double* T = P + s->panel_off[j];
            i32 ldj = s->stride[j];
            for (i32 q = 0; q < nf; q++) {
                i32 gc = grow[rs + q];
                i32 tc = gc - s->fcol[j];
                for (i32 i = 0; i < m; i++) {
                    i32 gr = grow[rs + i];
                    if (gr < gc) continue;
                    i32 pos = row_pos(s, j, gr);
                    if (pos < 0) { free(W); free(grow); return ORC_EINVAL; }
                    T[(i64)tc * ldj + pos] -= W[i + (i64)q * m];
                }
            }
            b = b2;
        }
    }
    free(W);
    free(grow);
    return ORC_OK;
}

/*
 * x = A^{-1} b with an L D L^T factor: permute, forward sweep with the unit
 * lower L, division by D, backward sweep with L^T, permute back.
 */
int orc_solve_ldlt(const orc_sym* s, const double* P, i32 nrhs, const double* B, i64 ldb, double* X, i64 ldx)
{
    double* Y = (double*)malloc(sizeof(double) * (size_t)s->n * (size_t)(nrhs > 0 ? nrhs : 1) + 8);
    if (!Y) return ORC_ENOMEM;
    for (i32 r = 0; r < nrhs; r++)
        for (i32 i = 0; i < s->n; i++) Y[(i64)r * s->n + i] = B[(i64)r * ldb + s->perm[i]];
    for (i32 rhs = 0; rhs < nrhs; rhs++) {
        double* y = Y + (i64)rhs * s->n;
        for (i32 k = 0; k < s->ncblk; k++) {
            i32 wd = s->lcol[k] - s->fcol[k] + 1, ld = s->stride[k], f = s->fcol[k];
            const double* L = P + s->panel_off[k];
            for (i32 c = 0; c < wd; c++) {
                double v = y[f + c];
                for (i32 p = 0; p < c; p++) v -= L[c + (i64)p * ld] * y[f + p];
                y[f + c] = v;
            }
            for (i32 b = s->bptr[k] + 1; b < s->bptr[k + 1]; b++)
                for (i32 r = s->frow[b]; r <= s->lrow[b]; r++) {
                    i32 pr = s->coefind[b] + r - s->frow[b];
                    double acc = 0.0;
                    for (i32 c = 0; c < wd; c++) acc += L[pr + (i64)c * ld] * y[f + c];
                    y[r] -= acc;
                }
        }
        for (i32 k = 0; k < s->ncblk; k++) {
            i32 wd = s->lcol[k] - s->fcol[k] + 1, ld = s->stride[k], f = s->fcol[k];
            const double* L = P + s->panel_off[k];
            for (i32 c = 0; c < wd; c++) y[f + c] /= L[c + (i64)c * ld];
        }
        for (i32 k = s->ncblk - 1; k >= 0; k--) {
            i32 wd = s->lcol[k] - s->fcol[k] + 1, ld = s->stride[k], f = s->fcol[k];
            const double* L = P + s->panel_off[k];
            for (i32 c = 0; c < wd; c++) {
                double acc = 0.0;
                for (i32 b = s->bptr[k] + 1; b < s->bptr[k + 1]; b++)
                    for (i32 r = s->frow[b]; r <= s->lrow[b]; r++)
                        acc += L[s->coefind[b] + r - s->frow[b] + (i64)c * ld] * y[r];
                y[f + c] -= acc;
            }
            for (i32 c = wd - 1; c >= 0; c--) {
                double v = y[f + c];
                for (i32 p = c + 1; p < wd; p++) v -= L[p + (i64)c * ld] * y[f + p];
                y[f + c] = v;
            }
        }
    }
    for (i32 r = 0; r < nrhs; r++)
        for (i32 i = 0; i < s->n; i++) X[(i64)r * ldx + s->perm[i]] = Y[(i64)r * s->n + i];
    free(Y);
    return ORC_OK;
}

/* log |det A| = sum log |d_j| (pairwise) and the number of negative pivots. */
static double pairwise(const double* v, i64 n);
double orc_logabsdet_ldlt(const orc_sym* s, const double* P, i32* nneg)
{
    double* t = (double*)malloc(sizeof(double) * ((size_t)s->n + 1));
    *nneg = 0;
    for (i32 k = 0; k < s->ncblk; k++) {
        i32 wd = s->lcol[k] - s->fcol[k] + 1, ld = s->stride[k];
        for (i32 c = 0; c < wd; c++) {
            double d = P[s->panel_off[k] + c + (i64)c * ld];
            if (d < 0.0) (*nneg)++;
            t[s->fcol[k] + c] = log(fabs(d));
        }
    }
    double r = pairwise(t, s->n);
    free(t);
    return r;
}

/*
 * L U with static pivoting (Section III: the solver works on the pattern of
 * A + A^T and, for a non-symmetric matrix, duplicates steps 2 and 3 for L
 * and U; no dynamic pivoting).  Two panel arrays with the layout of the
 * Cholesky factor:
 *   PL: the square diagonal block holds L_kk (strictly lower, unit diagonal
 *       implied) and U_kk (upper, diagonal included); the rows below hold
 *       L_off;
 *   PU: the rows below the diagonal block hold U_off^T (row r, column c is
 *       U(c, r)); its diagonal block is not used.
 * Assembly: an entry a_ij (permuted a, b) with a >= b goes to PL (column b,
 * row a); with a < b to PL's diagonal block (row a, column b) when both are
 * in one column block, else to PU (column a, row b).
 */
int orc_assemble_lu(const orc_sym* s, const i64* colptr, const i32* rowind, const double* val, double* PL,
                    double* PU)
{
    memset(PL, 0, sizeof(double) * (size_t)s->panel_size);
    memset(PU, 0, sizeof(double) * (size_t)s->panel_size);
    i32* col2cblk = (i32*)malloc(sizeof(i32) * ((size_t)s->n + 1));
    for (i32 k = 0; k < s->ncblk; k++) for (i32 j = s->fcol[k]; j <= s->lcol[k]; j++) col2cblk[j] = k;
    for (i32 j = 0; j < s->n; j++)
        for (i64 p = colptr[j]; p < colptr[j + 1]; p++) {
            i32 a = s->iperm[rowind[p]], b = s->iperm[j];
            if (a >= b) {
                i32 k = col2cblk[b], pos = row_pos(s, k, a);
                if (pos < 0) { free(col2cblk); return ORC_EINVAL; }
                PL[s->panel_off[k] + (i64)(b - s->fcol[k]) * s->stride[k] + pos] += val[p];
            } else {
                i32 k = col2cblk[a];
                if (b <= s->lcol[k]) {
                    PL[s->panel_off[k] + (i64)(b - s->fcol[k]) * s->stride[k] + (a - s->fcol[k])] += val[p];
                } else {
                    i32 pos = row_pos(s, k, b);
                    if (pos < 0) { free(col2cblk); return ORC_EINVAL; }
                    PU[s->panel_off[k] + (i64)(a - s->fcol[k]) * s->stride[k] + pos] += val[p];
                }
            }
        }
    free(col2cblk);
    return ORC_OK;
}

/*
 * Right-looking supernodal L U in ascending column-block order:
 *   1. L U of the square diagonal block (no pivoting); breakdown when a
 *      pivot is zero or not finite;
 *   2. L_off = A_off U_kk^{-1} (rows of PL below the block) and
 *      U_off = L_kk^{-1} A_upper (rows of PU: columns of U to the right);
 *   3. for every facing column block j: the rows of k from the first block
 *      facing j on (i) and the facing rows (q): W_L = L_rows U_facing and
 *      W_U = U_rows^T L_facing^T; the square part (both in j's diagonal
 *      block) is subtracted from PL's diagonal block of j in full, the rows
 *      beyond it from PL (W_L) and PU (W_U) of j.
 */
int orc_factor_lu_sp(const orc_sym* s, double* PL, double* PU, double tau, i32* nrep, i32* fail_col);

int orc_factor_lu(const orc_sym* s, double* PL, double* PU, i32* fail_col)
{
    i32 nrep = 0;
    return orc_factor_lu_sp(s, PL, PU, 0.0, &nrep, fail_col);
}

/* L U with the static pivot replacement of orc_factor_ldlt_sp (the pivot
 * u_cc replaced in place before it is used). */
int orc_factor_lu_sp(const orc_sym* s, double* PL, double* PU, double tau, i32* nrep, i32* fail_col)
{
    *fail_col = -1;
    *nrep = 0;
    i32 maxs = 0;
    for (i32 k = 0; k < s->ncblk; k++) if (s->stride[k] > maxs) maxs = s->stride[k];
    double* WL = (double*)malloc(sizeof(double) * (size_t)maxs * (size_t)maxs + 8);
    double* WU = (double*)malloc(sizeof(double) * (size_t)maxs * (size_t)maxs + 8);
    i32* grow = (i32*)malloc(sizeof(i32) * ((size_t)maxs + 1));
    if (!WL || !WU || !grow) return ORC_ENOMEM;
    for (i32 k = 0; k < s->ncblk; k++) {
        i32 wd = s->lcol[k] - s->fcol[k] + 1, ld = s->stride[k];
        double* L = PL + s->panel_off[k];
        double* U = PU + s->panel_off[k];
        for (i32 b = s->bptr[k]; b < s->bptr[k + 1]; b++)
            for (i32 r = s->frow[b]; r <= s->lrow[b]; r++) grow[s->coefind[b] + r - s->frow[b]] = r;
        /* 1. diagonal block, in place (B(r, c) at L[r + c*ld]) */
        for (i32 c = 0; c < wd; c++) {
            double d = static_pivot(L[c + (i64)c * ld], tau, nrep);
            L[c + (i64)c * ld] = d;
            if (!(d != 0.0) || !isfinite(d)) {
                *fail_col = s->fcol[k] + c;
                free(WL); free(WU); free(grow);
                return ORC_ENOTPD;
            }
            for (i32 r = c + 1; r < wd; r++) L[r + (i64)c * ld] /= d;
            for (i32 q = c + 1; q < wd; q++)
                for (i32 r = c + 1; r < wd; r++) L[r + (i64)q * ld] -= L[r + (i64)c * ld] * L[c + (i64)q * ld];
        }
        /* 2. rows below: L_off against U_kk (upper), U_off^T against L_kk (unit lower) */
        for (i32 r = wd; r < ld; r++)
            for (i32 c = 0; c < wd; c++) {
                double v = L[r + (i64)c * ld];
                for (i32 p = 0; p < c; p++) v -= L[r + (i64)p * ld] * L[p + (i64)c * ld];
                L[r + (i64)c * ld] = v / L[c + (i64)c * ld];
                double u = U[r + (i64)c * ld];
                for (i32 p = 0; p < c; p++) u -= L[c + (i64)p * ld] * U[r + (i64)p * ld];
                U[r + (i64)c * ld] = u;
            }
        /* 3. updates of the facing panels */
        for (i32 b = s->bptr[k] + 1; b < s->bptr[k + 1];) {
            i32 j = s->fcblk[b];
            i32 b2 = b;
            while (b2 < s->bptr[k + 1] && s->fcblk[b2] == j) b2++;
            i32 rs = s->coefind[b];
            i32 nf = s->coefind[b2 - 1] + (s->lrow[b2 - 1] - s->frow[b2 - 1] + 1) - rs;
            i32 m = ld - rs;
            for (i32 q = 0; q < nf; q++)
                for (i32 i = 0; i < m; i++) {
                    double al = 0.0, au = 0.0;
                    for (i32 p = 0; p < wd; p++) {
                        al += L[rs + i + (i64)p * ld] * U[rs + q + (i64)p * ld];
                        au += U[rs + i + (i64)p * ld] * L[rs + q + (i64)p * ld];
                    }
                    WL[i + (i64)q * m] = al;
                    WU[i + (i64)q * m] = au;
                }
            double* TL = PL + s->panel_off[j];
            double* TU = PU + s->panel_off[j];
            i32 ldj = s->stride[j];
            for (i32 q = 0; q < nf; q++) {
                i32 gc = grow[rs + q];
                i32 tc = gc - s->fcol[j];
                for (i32 i = 0; i < m; i++) {
                    i32 gr = grow[rs + i];
                    if (gr <= s->lcol[j]) {   /* both in j's diagonal block: (row gr, column gc) */
                        TL[(i64)tc * ldj + (gr - s->fcol[j])] -= WL[i + (i64)q * m];
                        continue;
                    }
                    i32 pos = row_pos(s, j, gr);
                    if (pos < 0) { free(WL); free(WU); free(grow); return ORC_EINVAL; }
                    TL[(i64)tc * ldj + pos] -= WL[i + (i64)q * m];
                    TU[(i64)tc * ldj + pos] -= WU[i + (i64)q * m];
                }
            }
            b = b2;
        }
    }
    free(WL);
    free(WU);
    free(grow);
    return ORC_OK;
}

/* x = A^{-1} b with an L U factor: permute, forward sweep with the unit lower
 * L, backward sweep with U (diagonal blocks in PL, the rest in PU),
 * permute back. */
int orc_solve_lu(const orc_sym* s, const double* PL, const double* PU, i32 nrhs, const double* B, i64 ldb,
                 double* X, i64 ldx)
{
    double* Y = (double*)malloc(sizeof(double) * (size_t)s->n * (size_t)(nrhs > 0 ? nrhs : 1) + 8);
    if (!Y) return ORC_ENOMEM;
    for (i32 r = 0; r < nrhs; r++)
        for (i32 i = 0; i < s->n; i++) Y[(i64)r * s->n + i] = B[(i64)r * ldb + s->perm[i]];
    for (i32 rhs = 0; rhs < nrhs; rhs++) {
        double* y = Y + (i64)rhs * s->n;
        for (i32 k = 0; k < s->ncblk; k++) {
            i32 wd = s->lcol[k] - s->fcol[k] + 1, ld = s->stride[k], f = s->fcol[k];
            const double* L = PL + s->panel_off[k];
            for (i32 c = 0; c < wd; c++) {
                double v = y[f + c];
                for (i32 p = 0; p < c; p++) v -= L[c + (i64)p * ld] * y[f + p];
                y[f + c] = v;
            }
            for (i32 b = s->bptr[k] + 1; b < s->bptr[k + 1]; b++)
                for (i32 r = s->frow[b]; r <= s->lrow[b]; r++) {
                    i32 pr = s->coefind[b] + r - s->frow[b];
                    double acc = 0.0;
                    for (i32 c = 0; c < wd; c++) acc += L[pr + (i64)c * ld] * y[f + c];
                    y[r] -= acc;
                }
        }
        for (i32 k = s->ncblk - 1; k >= 0; k--) {
            i32 wd = s->lcol[k] - s->fcol[k] + 1, ld = s->stride[k], f = s->fcol[k];
            const double* L = PL + s->panel_off[k];
            const double* U = PU + s->panel_off[k];
            for (i32 c = 0; c < wd; c++) {
                double acc = 0.0;
                for (i32 b = s->bptr[k] + 1; b < s->bptr[k + 1]; b++)
                    for (i32 r = s->frow[b]; r <= s->lrow[b]; r++)
                        acc += U[s->coefind[b] + r - s->frow[b] + (i64)c * ld] * y[r];
                y[f + c] -= acc;
            }
            for (i32 c = wd - 1; c >= 0; c--) {
                double v = y[f + c];
                for (i32 q = c + 1; q < wd; q++) v -= L[c + (i64)q * ld] * y[f + q];
                y[f + c] = v / L[c + (i64)c * ld];
            }
        }
    }
    for (i32 r = 0; r < nrhs; r++)
        for (i32 i = 0; i < s->n; i++) X[(i64)r * ldx + s->perm[i]] = Y[(i64)r * s->n + i];
    free(Y);
    return ORC_OK;
}

/* log |det A| = sum log |u_jj| (pairwise) and the number of negative u_jj. */
double orc_logabsdet_lu(const orc_sym* s, const double* PL, i32* nneg)
{
    return orc_logabsdet_ldlt(s, PL, nneg);
}

/*
 * Solve L L^T y = c in the final numbering, in place, for nrhs columns of
 * length n with leading dimension ldy.  Forward sweep in ascending block
 * order (diagonal solve, then subtract the off-diagonal products from the
 * facing rows), backward sweep in descending order with the transposes.
 */
int orc_solve_perm(const orc_sym* s, const double* P, i32 nrhs, double* Y, i64 ldy)
{
    for (i32 rhs = 0; rhs < nrhs; rhs++) {
        double* y = Y + (i64)rhs * ldy;
        for (i32 k = 0; k < s->ncblk; k++) {
            i32 wd = s->lcol[k] - s->fcol[k] + 1, ld = s->stride[k], f = s->fcol[k];
            const double* L = P + s->panel_off[k];
            for (i32 c = 0; c < wd; c++) {
                double v = y[f + c];
                for (i32 p = 0; p < c; p++) v -= L[c + (i64)p * ld] * y[f + p];
                y[f + c] = v / L[c + (i64)c * ld];
            }
            for (i32 b = s->bptr[k] + 1; b < s->bptr[k + 1]; b++)
                for (i32 r = s->frow[b]; r <= s->lrow[b]; r++) {
                    i32 pr = s->coefind[b] + r - s->frow[b];
                    double acc = 0.0;
                    for (i32 c = 0; c < wd; c++) acc += L[pr + (i64)c * ld] * y[f + c];
                    y[r] -= acc;
                }
        }
        for (i32 k = s->ncblk - 1; k >= 0; k--) {
            i32 wd = s->lcol[k] - s->fcol[k] + 1, ld = s->stride[k], f = s->fcol[k];
            const double* L = P + s->panel_off[k];
            for (i32 c = 0; c < wd; c++) {
                double acc = 0.0;
                for (i32 b = s->bptr[k] + 1; b < s->bptr[k + 1]; b++)
                    for (i32 r = s->frow[b]; r <= s->lrow[b]; r++)
                        acc += L[s->coefind[b] + r - s->frow[b] + (i64)c * ld] * y[r];
                y[f + c] -= acc;
            }
            for (i32 c = wd - 1; c >= 0; c--) {
                double v = y[f + c];
                for (i32 p = c + 1; p < wd; p++) v -= L[p + (i64)c * ld] * y[f + p];
                y[f + c] = v / L[c + (i64)c * ld];
            }
        }
    }
    return ORC_OK;
}

/* x = A^{-1} b with the factor: permute, solve, permute back. */
int orc_solve(const orc_sym* s, const double* P, i32 nrhs, const double* B, i64 ldb, double* X, i64 ldx)
{
    double* y = (double*)malloc(sizeof(double) * (size_t)s->n * (size_t)(nrhs > 0 ? nrhs : 1) + 8);
    for (i32 r = 0; r < nrhs; r++)
        for (i32 i = 0; i < s->n; i++) y[(i64)r * s->n + i] = B[(i64)r * ldb + s->perm[i]];
    orc_solve_perm(s, P, nrhs, y, s->n);
    for (i32 r = 0; r < nrhs; r++)
        for (i32 i = 0; i < s->n; i++) X[(i64)r * ldx + s->perm[i]] = y[(i64)r * s->n + i];
    free(y);
    return ORC_OK;
}

/*
 * r = b - A x and s = |A| |x| + |b| using the lower triangle of A mirrored
 * (entries with row >= col), as the factorization reads it.
 */
void orc_residual(i32 n, const i64* colptr, const i32* rowind, const double* val,
                  const double* x, const double* b, double* r, double* sden)
{
    for (i32 i = 0; i < n; i++) { r[i] = b[i]; sden[i] = fabs(b[i]); }
    for (i32 j = 0; j < n; j++)
        for (i64 p = colptr[j]; p < colptr[j + 1]; p++) {
            i32 i = rowind[p];
            if (i < j) continue;
            double a = val[p];
            r[i] -= a * x[j];
            sden[i] += fabs(a) * fabs(x[j]);
            if (i != j) { r[j] -= a * x[i]; sden[j] += fabs(a) * fabs(x[i]); }
        }
}

/* Componentwise backward error (Oettli-Prager): max_i |r_i| / s_i, 0/0 = 0, p/0 = inf. */
double orc_omega(i32 n, const double* r, const double* sden)
{
    double om = 0.0;
    for (i32 i = 0; i < n; i++) {
        double a = fabs(r[i]), q;
        if (a == 0.0) q = 0.0;
        else if (sden[i] == 0.0) q = INFINITY;
        else q = a / sden[i];
        if (q > om || q != q) om = q;
    }
    return om;
}

/* Pairwise sum of 2*log(l_jj). */
static double pairwise(const double* v, i64 n)
{
    if (n <= 8) { double s = 0.0; for (i64 i = 0; i < n; i++) s += v[i]; return s; }
    i64 h = n / 2;
    return pairwise(v, h) + pairwise(v + h, n - h);
}

double orc_logdet(const orc_sym* s, const double* P)
{
    double* t = (double*)malloc(sizeof(double) * ((size_t)s->n + 1));
    for (i32 k = 0; k < s->ncblk; k++) {
        i32 wd = s->lcol[k] - s->fcol[k] + 1, ld = s->stride[k];
        for (i32 c = 0; c < wd; c++) t[s->fcol[k] + c] = 2.0 * log(P[s->panel_off[k] + c + (i64)c * ld]);
    }
    double r = pairwise(t, s->n);
    free(t);
    return r;
}

/* Factor as coordinate triplets (final numbering), lower triangle only. */
i64 orc_unpack(const orc_sym* s, const double* P, i32* ri, i32* ci, double* v)
{
    i64 q = 0;
    for (i32 k = 0; k < s->ncblk; k++) {
        i32 wd = s->lcol[k] - s->fcol[k] + 1, ld = s->stride[k];
        const double* L = P + s->panel_off[k];
        for (i32 c = 0; c < wd; c++) {
            for (i32 r = c; r < wd; r++) { ri[q] = s->fcol[k] + r; ci[q] = s->fcol[k] + c; v[q] = L[r + (i64)c * ld]; q++; }
            for (i32 b = s->bptr[k] + 1; b < s->bptr[k + 1]; b++)
                for (i32 r = s->frow[b]; r <= s->lrow[b]; r++) {
                    ri[q] = r; ci[q] = s->fcol[k] + c; v[q] = L[s->coefind[b] + r - s->frow[b] + (i64)c * ld]; q++;
                }
        }
    }
    return q;
}

/*
 * Value gradient of a loss through x = A^{-1} b, A symmetric and given by
 * its lower triangle, from x and db = A^{-T} xbar (n x nrhs, column-major,
 * leading dimension ld).  The derivative with respect to the matrix is
 * dA = -db x^T summed over the right-hand sides; a stored entry (i, j) with
 * i > j sets both A_ij and A_ji, so it gets -sum_k (db_ik x_jk + db_jk x_ik);
 * a diagonal entry gets -sum_k db_ik x_ik; an entry above the diagonal is
 * never read and gets 0.
 */
void orc_values_grad(i32 n, const i64* colptr, const i32* rowind, i32 nrhs, const double* x, const double* db,
                     i64 ld, double* g)
{
    for (i32 j = 0; j < n; j++)
        for (i64 p = colptr[j]; p < colptr[j + 1]; p++) {
            i32 i = rowind[p];
            double acc = 0.0;
            if (i == j)
                for (i32 k = 0; k < nrhs; k++) acc += db[(i64)k * ld + i] * x[(i64)k * ld + i];
            else if (i > j)
                for (i32 k = 0; k < nrhs; k++)
                    acc += db[(i64)k * ld + i] * x[(i64)k * ld + j] + db[(i64)k * ld + j] * x[(i64)k * ld + i];
            g[p] = i < j ? 0.0 : -acc;
        }
}
