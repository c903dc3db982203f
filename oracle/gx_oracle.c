/*
 * gx_oracle.c -- plain FP64 CPU oracle for the N-body/SPH interaction path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant generator with the HIP path; it reads the same
 * seeded inputs and nothing the GPU wrote.
 *
 * Everything is double precision and deliberately unblocked: loops follow the
 * definitions so a reader can check them against the paper by eye.
 *
 *   gravity   Eq. 1 (softened pairwise law, Sec. 3.5), potential = the
 *             matching softened Plummer potential, self pair excluded.
 *   tree      Barnes-Hut octree over Morton-sorted particles (Sec. 3.4),
 *             groups of at most n_g particles sharing one interaction list
 *             (Sec. 5.2.2 / 5.2.4), opening criterion l_c < theta * d_min,
 *             monopole + traceless quadrupole cells.
 *   SPH       Wendland C4 kernel, kernel size solved from
 *             (4 pi / 3) H^3 rho / m = N_ngb by safeguarded Newton (the
 *             "kernel size calculation" of Sec. 5.2.5 / Table 3), density,
 *             pressure, symmetric pressure-gradient force with
 *             signal-velocity artificial viscosity (Table 3 / Table 4 kernels).
 *
 * The paper never writes its SPH equations, its quadrupole or its opening
 * criterion; the forms used here are the readings listed in the project's
 * design notes.  Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC.
 * FP contraction is off so the key and opening-criterion arithmetic is the
 * exact IEEE sequence written below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_API __attribute__((visibility("default")))
#define KEY_BITS 21
#define MAX_LEVEL 21

/* ------------------------------------------------------------------------ */
/* 1. Direct-sum gravity, Eq. 1                                              */
/* ------------------------------------------------------------------------ */

/* a_i = -G sum_{j != i} m_j (r_i - r_j) / (|r_i - r_j|^2 + eps_i^2 + eps_j^2)^{3/2}
 * phi_i = -G sum_{j != i} m_j / (|r_i - r_j|^2 + eps_i^2 + eps_j^2)^{1/2}
 * Receivers: idx[0..ni) (original indices), or all n when idx == NULL.
 * Outputs are indexed by receiver slot k (0..ni). */
ORC_API void orc_direct_gravity(int64_t n, const double* x, const double* y, const double* z,
                                const double* m, const double* eps2, double G, int64_t ni,
                                const int64_t* idx, double* ax, double* ay, double* az,
                                double* pot) {
    int64_t nrecv = idx ? ni : n;
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t k = 0; k < nrecv; k++) {
        int64_t i = idx ? idx[k] : k;
        double sx = 0, sy = 0, sz = 0, sp = 0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            double rx = x[i] - x[j], ry = y[i] - y[j], rz = z[i] - z[j];
            double r2 = rx * rx + ry * ry + rz * rz + eps2[i] + eps2[j];
            double rinv = 1.0 / sqrt(r2);
            double rinv3 = rinv * rinv * rinv;
            sx -= m[j] * rx * rinv3;
            sy -= m[j] * ry * rinv3;
            sz -= m[j] * rz * rinv3;
            sp -= m[j] * rinv;
        }
        ax[k] = G * sx;
        ay[k] = G * sy;
        az[k] = G * sz;
        pot[k] = G * sp;
    }
}

/* ------------------------------------------------------------------------ */
/* 2. Morton-ordered octree                                                  */
/* ------------------------------------------------------------------------ */

typedef struct orc_tree {
    int64_t n;
    int n_leaf, n_group;
    double x0[3], L, scale; /* root corner, root side, 2^21 / L */
    uint64_t* key;          /* sorted keys */
    int64_t* perm;          /* sorted slot -> original index */
    double *xs, *ys, *zs, *ms, *e2s;
    /* nodes, depth-first pre-order, children in Morton order */
    int64_t nn, cap;
    int64_t *nb, *ne, *next;
    int32_t* lev;
    int8_t* leaf;
    double *mass, *com, *quad, *e2bar, *lo, *hi, *hmax;
    int64_t ng;
    int64_t* gnode; /* node id of each group, in pre-order */
} orc_tree;

typedef struct {
    uint64_t k;
    int64_t i;
} kv_t;

static int kv_cmp(const void* a, const void* b) {
    const kv_t* p = (const kv_t*)a;
    const kv_t* q = (const kv_t*)b;
    if (p->k != q->k) return p->k < q->k ? -1 : 1;
    return p->i < q->i ? -1 : (p->i > q->i); /* ties keep input order: a stable sort */
}

/* Spread the low 21 bits of v so bit b moves to bit 3b. */
static uint64_t spread3(uint64_t v) {
    uint64_t r = 0;
    for (int b = 0; b < KEY_BITS; b++) r |= ((v >> b) & 1ull) << (3 * b);
    return r;
}

/* Integer cell coordinate of one axis: min(2^21 - 1, floor((x - x0) * scale)). */
static uint64_t axis_cell(double x, double x0, double scale) {
    double t = (x - x0) * scale;
    double f = floor(t);
    if (f > 2097151.0) f = 2097151.0;
    if (f < 0.0) f = 0.0;
    return (uint64_t)f;
}

static uint64_t morton_key(double x, double y, double z, const double* x0, double scale) {
    uint64_t ix = axis_cell(x, x0[0], scale), iy = axis_cell(y, x0[1], scale),
             iz = axis_cell(z, x0[2], scale);
    return (spread3(ix) << 2) | (spread3(iy) << 1) | spread3(iz);
}

ORC_API void orc_root_box(int64_t n, const double* x, const double* y, const double* z,
                          double* out4 /* x0, y0, z0, L */) {
    double mn[3] = {x[0], y[0], z[0]}, mx[3] = {x[0], y[0], z[0]};
    for (int64_t i = 1; i < n; i++) {
        const double p[3] = {x[i], y[i], z[i]};
        for (int d = 0; d < 3; d++) {
            if (p[d] < mn[d]) mn[d] = p[d];
            if (p[d] > mx[d]) mx[d] = p[d];
        }
    }
    double ext = 0.0;
    for (int d = 0; d < 3; d++)
        if (mx[d] - mn[d] > ext) ext = mx[d] - mn[d];
    if (ext == 0.0) ext = 1.0;
    out4[0] = mn[0];
    out4[1] = mn[1];
    out4[2] = mn[2];
    out4[3] = ext * (1.0 + 0x1p-40);
}

ORC_API void orc_morton_keys(int64_t n, const double* x, const double* y, const double* z,
                             const double* box4, uint64_t* keys) {
    double scale = 2097152.0 / box4[3];
    for (int64_t i = 0; i < n; i++) keys[i] = morton_key(x[i], y[i], z[i], box4, scale);
}

static int64_t push_node(orc_tree* T) {
    if (T->nn == T->cap) {
        int64_t c = T->cap ? 2 * T->cap : 1024;
        T->nb = realloc(T->nb, c * sizeof(int64_t));
        T->ne = realloc(T->ne, c * sizeof(int64_t));
        T->next = realloc(T->next, c * sizeof(int64_t));
        T->lev = realloc(T->lev, c * sizeof(int32_t));
        T->leaf = realloc(T->leaf, c * sizeof(int8_t));
        T->cap = c;
    }
    return T->nn++;
}

/* Depth-first construction: a node is split while it holds more than n_leaf
 * particles and is above the finest level; empty children are not created. */
static void build_node(orc_tree* T, int level, int64_t b, int64_t e) {
    int64_t id = push_node(T);
    T->nb[id] = b;
    T->ne[id] = e;
    T->lev[id] = level;
    if (e - b > T->n_leaf && level < MAX_LEVEL) {
        T->leaf[id] = 0;
        int shift = 3 * (MAX_LEVEL - (level + 1));
        int64_t s = b;
        for (uint64_t d = 0; d < 8; d++) {
            int64_t t = s;
            while (t < e && ((T->key[t] >> shift) & 7ull) == d) t++;
            if (t > s) build_node(T, level + 1, s, t);
            s = t;
        }
    } else {
        T->leaf[id] = 1;
    }
    T->next[id] = T->nn;
}

/* Moments of one node straight from its particles: mass, centre of mass,
 * traceless quadrupole Q_ab = sum m (3 d_a d_b - |d|^2 delta_ab) about the
 * centre of mass, mass-weighted mean eps^2, tight bounding box. */
static void node_moments(orc_tree* T, int64_t id) {
    int64_t b = T->nb[id], e = T->ne[id];
    double M = 0, cx = 0, cy = 0, cz = 0, e2 = 0;
    double lo[3] = {T->xs[b], T->ys[b], T->zs[b]}, hi[3] = {T->xs[b], T->ys[b], T->zs[b]};
    for (int64_t k = b; k < e; k++) {
        M += T->ms[k];
        cx += T->ms[k] * T->xs[k];
        cy += T->ms[k] * T->ys[k];
        cz += T->ms[k] * T->zs[k];
        e2 += T->ms[k] * T->e2s[k];
        const double p[3] = {T->xs[k], T->ys[k], T->zs[k]};
        for (int d = 0; d < 3; d++) {
            if (p[d] < lo[d]) lo[d] = p[d];
            if (p[d] > hi[d]) hi[d] = p[d];
        }
    }
    cx /= M;
    cy /= M;
    cz /= M;
    double q[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t k = b; k < e; k++) {
        double dx = T->xs[k] - cx, dy = T->ys[k] - cy, dz = T->zs[k] - cz;
        double d2 = dx * dx + dy * dy + dz * dz;
        double mk = T->ms[k];
        q[0] += mk * (3 * dx * dx - d2);
        q[1] += mk * (3 * dy * dy - d2);
        q[2] += mk * (3 * dz * dz - d2);
        q[3] += mk * 3 * dx * dy;
        q[4] += mk * 3 * dx * dz;
        q[5] += mk * 3 * dy * dz;
    }
    T->mass[id] = M;
    T->com[3 * id] = cx;
    T->com[3 * id + 1] = cy;
    T->com[3 * id + 2] = cz;
    for (int c = 0; c < 6; c++) T->quad[6 * id + c] = q[c];
    T->e2bar[id] = e2 / M;
    for (int d = 0; d < 3; d++) {
        T->lo[3 * id + d] = lo[d];
        T->hi[3 * id + d] = hi[d];
    }
}

static void collect_groups(orc_tree* T, int64_t id) {
    if (T->ne[id] - T->nb[id] <= T->n_group || T->leaf[id]) {
        T->gnode[T->ng++] = id;
        return;
    }
    for (int64_t c = id + 1; c < T->next[id]; c = T->next[c]) collect_groups(T, c);
}

ORC_API orc_tree* orc_tree_build(int64_t n, const double* x, const double* y, const double* z,
                                 const double* m, const double* eps2, int n_leaf, int n_group) {
    orc_tree* T = calloc(1, sizeof(orc_tree));
    T->n = n;
    T->n_leaf = n_leaf;
    T->n_group = n_group;
    double box[4];
    orc_root_box(n, x, y, z, box);
    T->x0[0] = box[0];
    T->x0[1] = box[1];
    T->x0[2] = box[2];
    T->L = box[3];
    T->scale = 2097152.0 / T->L;
    kv_t* kv = malloc(n * sizeof(kv_t));
    for (int64_t i = 0; i < n; i++) {
        kv[i].k = morton_key(x[i], y[i], z[i], T->x0, T->scale);
        kv[i].i = i;
    }
    qsort(kv, n, sizeof(kv_t), kv_cmp);
    T->key = malloc(n * sizeof(uint64_t));
    T->perm = malloc(n * sizeof(int64_t));
    T->xs = malloc(n * sizeof(double));
    T->ys = malloc(n * sizeof(double));
    T->zs = malloc(n * sizeof(double));
    T->ms = malloc(n * sizeof(double));
    T->e2s = malloc(n * sizeof(double));
    for (int64_t s = 0; s < n; s++) {
        int64_t i = kv[s].i;
        T->key[s] = kv[s].k;
        T->perm[s] = i;
        T->xs[s] = x[i];
        T->ys[s] = y[i];
        T->zs[s] = z[i];
        T->ms[s] = m[i];
        T->e2s[s] = eps2 ? eps2[i] : 0.0;
    }
    free(kv);
    build_node(T, 0, 0, n);
    int64_t nn = T->nn;
    T->mass = malloc(nn * sizeof(double));
    T->com = malloc(3 * nn * sizeof(double));
    T->quad = malloc(6 * nn * sizeof(double));
    T->e2bar = malloc(nn * sizeof(double));
    T->lo = malloc(3 * nn * sizeof(double));
    T->hi = malloc(3 * nn * sizeof(double));
    T->hmax = calloc(nn, sizeof(double));
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t id = 0; id < nn; id++) node_moments(T, id);
    T->gnode = malloc(nn * sizeof(int64_t));
    T->ng = 0;
    collect_groups(T, 0);
    return T;
}

ORC_API void orc_tree_free(orc_tree* T) {
    if (!T) return;
    free(T->key); free(T->perm); free(T->xs); free(T->ys); free(T->zs); free(T->ms);
    free(T->e2s); free(T->nb); free(T->ne); free(T->next); free(T->lev); free(T->leaf);
    free(T->mass); free(T->com); free(T->quad); free(T->e2bar); free(T->lo); free(T->hi);
    free(T->hmax); free(T->gnode); free(T);
}

ORC_API int64_t orc_tree_nnodes(const orc_tree* T) { return T->nn; }
ORC_API int64_t orc_tree_ngroups(const orc_tree* T) { return T->ng; }
ORC_API void orc_tree_box(const orc_tree* T, double* out4) {
    out4[0] = T->x0[0]; out4[1] = T->x0[1]; out4[2] = T->x0[2]; out4[3] = T->L;
}

ORC_API void orc_tree_get_sorted(const orc_tree* T, uint64_t* key, int64_t* perm) {
    memcpy(key, T->key, T->n * sizeof(uint64_t));
    memcpy(perm, T->perm, T->n * sizeof(int64_t));
}

ORC_API void orc_tree_get_nodes(const orc_tree* T, int64_t* nb, int64_t* ne, int64_t* next,
                                int32_t* lev, int8_t* leaf, double* mass, double* com,
                                double* quad, double* e2bar, double* lo, double* hi) {
    int64_t nn = T->nn;
    memcpy(nb, T->nb, nn * 8); memcpy(ne, T->ne, nn * 8); memcpy(next, T->next, nn * 8);
    memcpy(lev, T->lev, nn * 4); memcpy(leaf, T->leaf, nn);
    memcpy(mass, T->mass, nn * 8); memcpy(com, T->com, 3 * nn * 8);
    memcpy(quad, T->quad, 6 * nn * 8); memcpy(e2bar, T->e2bar, nn * 8);
    memcpy(lo, T->lo, 3 * nn * 8); memcpy(hi, T->hi, 3 * nn * 8);
}

ORC_API void orc_tree_get_groups(const orc_tree* T, int64_t* gnode) {
    memcpy(gnode, T->gnode, T->ng * 8);
}

/* Squared minimum distance between two axis-aligned boxes, written as the
 * exact IEEE sequence used by the opening criterion. */
static double box_d2(const double* alo, const double* ahi, const double* blo, const double* bhi) {
    double s = 0.0;
    for (int d = 0; d < 3; d++) {
        double t1 = blo[d] - ahi[d];
        double t2 = alo[d] - bhi[d];
        double t = t1 > t2 ? t1 : t2;
        if (t < 0.0) t = 0.0;
        double tt = t * t;
        s = s + tt;
    }
    return s;
}

/* Interaction list of group g: cells accepted by l_c^2 < theta^2 d_min^2 go
 * to the cell (pc) list; rejected leaves go to the particle (pp) list as node
 * ids; rejected internal nodes are opened.  mode 0 counts, mode 1 fills. */
static void walk_group(const orc_tree* T, int64_t g, double theta2, int64_t* npp_leaf,
                       int64_t* npc, int64_t* npp_part, int64_t* pp_out, int64_t* pc_out) {
    int64_t gid = T->gnode[g];
    const double* glo = &T->lo[3 * gid];
    const double* ghi = &T->hi[3 * gid];
    int64_t a = 0, c = 0, p = 0;
    for (int64_t node = 0; node < T->nn;) {
        double d2 = box_d2(glo, ghi, &T->lo[3 * node], &T->hi[3 * node]);
        double lc = ldexp(T->L, -T->lev[node]);
        double lhs = lc * lc;
        double rhs = theta2 * d2;
        if (lhs < rhs) {
            if (pc_out) pc_out[c] = node;
            c++;
            node = T->next[node];
        } else if (T->leaf[node]) {
            if (pp_out) pp_out[a] = node;
            a++;
            p += T->ne[node] - T->nb[node];
            node = T->next[node];
        } else {
            node = node + 1;
        }
    }
    *npp_leaf = a;
    *npc = c;
    *npp_part = p;
}

/* Per-group counts: pp leaves, pc cells, pp particles. */
ORC_API void orc_tree_list_counts(const orc_tree* T, double theta, int64_t* npp_leaf,
                                  int64_t* npc, int64_t* npp_part) {
    double theta2 = theta * theta;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t g = 0; g < T->ng; g++)
        walk_group(T, g, theta2, &npp_leaf[g], &npc[g], &npp_part[g], NULL, NULL);
}

/* Fill CSR lists given offsets from the counts (leaf node ids and cell ids). */
ORC_API void orc_tree_list_fill(const orc_tree* T, double theta, const int64_t* pp_off,
                                const int64_t* pc_off, int64_t* pp_leaf, int64_t* pc_node) {
    double theta2 = theta * theta;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t g = 0; g < T->ng; g++) {
        int64_t a, c, p;
        walk_group(T, g, theta2, &a, &c, &p, pp_leaf + pp_off[g], pc_node + pc_off[g]);
    }
}

/* Tree gravity in FP64: for each receiver in each group, the exact pair law
 * over the particles of every listed leaf (self excluded), plus for every
 * accepted cell the monopole and, when quad != 0, the quadrupole term
 *   phi += -G [M/R + r.Q.r / (2 R^5)],
 *   a   += -G [M r / R^3 - Q r / R^5 + (5/2) (r.Q.r) r / R^7],
 * with r = r_i - s (s = centre of mass) and R^2 = |r|^2 + eps_i^2 + mean eps_c^2.
 * Results are written at original particle indices. */
/* Gravity for the receivers of the listed groups (all groups when gsel is
 * NULL); outputs at original indices.  Returns interaction counts. */
static void tree_gravity_groups(const orc_tree* T, double G, double theta, int quad,
                                int64_t ngs, const int64_t* gsel, double* ax, double* ay,
                                double* az, double* pot, int64_t* n_pp_out, int64_t* n_pc_out) {
    double theta2 = theta * theta;
    int64_t tot_pp = 0, tot_pc = 0;
    int64_t nsel = gsel ? ngs : T->ng;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : tot_pp, tot_pc)
    for (int64_t k = 0; k < nsel; k++) {
        int64_t g = gsel ? gsel[k] : k;
        int64_t a, c, p;
        walk_group(T, g, theta2, &a, &c, &p, NULL, NULL);
        int64_t* leaves = malloc((a + 1) * sizeof(int64_t));
        int64_t* cells = malloc((c + 1) * sizeof(int64_t));
        walk_group(T, g, theta2, &a, &c, &p, leaves, cells);
        int64_t gid = T->gnode[g];
        for (int64_t s = T->nb[gid]; s < T->ne[gid]; s++) {
            double xi = T->xs[s], yi = T->ys[s], zi = T->zs[s], e2i = T->e2s[s];
            double sx = 0, sy = 0, sz = 0, sp = 0;
            for (int64_t l = 0; l < a; l++) {
                int64_t nd = leaves[l];
                for (int64_t j = T->nb[nd]; j < T->ne[nd]; j++) {
                    if (j == s) continue;
                    double rx = xi - T->xs[j], ry = yi - T->ys[j], rz = zi - T->zs[j];
                    double r2 = rx * rx + ry * ry + rz * rz + e2i + T->e2s[j];
                    double rinv = 1.0 / sqrt(r2);
                    double rinv3 = rinv * rinv * rinv;
                    sx -= T->ms[j] * rx * rinv3;
                    sy -= T->ms[j] * ry * rinv3;
                    sz -= T->ms[j] * rz * rinv3;
                    sp -= T->ms[j] * rinv;
                }
            }
            for (int64_t l = 0; l < c; l++) {
                int64_t nd = cells[l];
                double M = T->mass[nd];
                double rx = xi - T->com[3 * nd], ry = yi - T->com[3 * nd + 1],
                       rz = zi - T->com[3 * nd + 2];
                double R2 = rx * rx + ry * ry + rz * rz + e2i + T->e2bar[nd];
                double Rinv = 1.0 / sqrt(R2);
                double Rinv2 = Rinv * Rinv;
                double Rinv3 = Rinv * Rinv2;
                sx -= M * rx * Rinv3;
                sy -= M * ry * Rinv3;
                sz -= M * rz * Rinv3;
                sp -= M * Rinv;
                if (quad) {
                    const double* Q = &T->quad[6 * nd];
                    double Qrx = Q[0] * rx + Q[3] * ry + Q[4] * rz;
                    double Qry = Q[3] * rx + Q[1] * ry + Q[5] * rz;
                    double Qrz = Q[4] * rx + Q[5] * ry + Q[2] * rz;
                    double rQr = rx * Qrx + ry * Qry + rz * Qrz;
                    double Rinv5 = Rinv3 * Rinv2;
                    double Rinv7 = Rinv5 * Rinv2;
                    sx -= -Qrx * Rinv5 + 2.5 * rQr * rx * Rinv7;
                    sy -= -Qry * Rinv5 + 2.5 * rQr * ry * Rinv7;
                    sz -= -Qrz * Rinv5 + 2.5 * rQr * rz * Rinv7;
                    sp -= 0.5 * rQr * Rinv5;
                }
            }
            int64_t i = T->perm[s];
            ax[i] = G * sx;
            ay[i] = G * sy;
            az[i] = G * sz;
            pot[i] = G * sp;
        }
        tot_pp += p * (T->ne[gid] - T->nb[gid]);
        tot_pc += c * (T->ne[gid] - T->nb[gid]);
        free(leaves);
        free(cells);
    }
    if (n_pp_out) *n_pp_out = tot_pp;
    if (n_pc_out) *n_pc_out = tot_pc;
}

/* Tree gravity in FP64: for each receiver in each group, the exact pair law
 * over the particles of every listed leaf (self excluded), plus for every
 * accepted cell the monopole and, when quad != 0, the quadrupole term
 *   phi += -G [M/R + r.Q.r / (2 R^5)],
 *   a   += -G [M r / R^3 - Q r / R^5 + (5/2) (r.Q.r) r / R^7],
 * with r = r_i - s (s = centre of mass) and R^2 = |r|^2 + eps_i^2 + mean eps_c^2.
 * Results are written at original particle indices. */
ORC_API void orc_tree_gravity(const orc_tree* T, double G, double theta, int quad, double* ax,
                              double* ay, double* az, double* pot, int64_t* n_pp_out,
                              int64_t* n_pc_out) {
    tree_gravity_groups(T, G, theta, quad, 0, NULL, ax, ay, az, pot, n_pp_out, n_pc_out);
}

/* The same for a subset of groups (a bounded sample of a large workload). */
ORC_API void orc_tree_gravity_groups(const orc_tree* T, double G, double theta, int quad,
                                     int64_t ngs, const int64_t* gsel, double* ax, double* ay,
                                     double* az, double* pot, int64_t* n_pp_out,
                                     int64_t* n_pc_out) {
    tree_gravity_groups(T, G, theta, quad, ngs, gsel, ax, ay, az, pot, n_pp_out, n_pc_out);
}

/* Potential and acceleration at point r from one node's multipole expansion
 * (monopole, plus quadrupole when quad != 0), unsoftened; used to check the
 * expansion's order of accuracy against the direct sum over its members. */
ORC_API void orc_node_field(const orc_tree* T, int64_t node, int quad, const double* r,
                            double* out4) {
    double M = T->mass[node];
    double rx = r[0] - T->com[3 * node], ry = r[1] - T->com[3 * node + 1],
           rz = r[2] - T->com[3 * node + 2];
    double R2 = rx * rx + ry * ry + rz * rz;
    double Rinv = 1.0 / sqrt(R2), Rinv2 = Rinv * Rinv, Rinv3 = Rinv * Rinv2;
    double a[3] = {-M * rx * Rinv3, -M * ry * Rinv3, -M * rz * Rinv3};
    double p = -M * Rinv;
    if (quad) {
        const double* Q = &T->quad[6 * node];
        double Qr[3] = {Q[0] * rx + Q[3] * ry + Q[4] * rz, Q[3] * rx + Q[1] * ry + Q[5] * rz,
                        Q[4] * rx + Q[5] * ry + Q[2] * rz};
        double rQr = rx * Qr[0] + ry * Qr[1] + rz * Qr[2];
        double Rinv5 = Rinv3 * Rinv2, Rinv7 = Rinv5 * Rinv2;
        const double rr[3] = {rx, ry, rz};
        for (int d = 0; d < 3; d++) a[d] -= -Qr[d] * Rinv5 + 2.5 * rQr * rr[d] * Rinv7;
        p -= 0.5 * rQr * Rinv5;
    }
    out4[0] = a[0];
    out4[1] = a[1];
    out4[2] = a[2];
    out4[3] = p;
}

/* ------------------------------------------------------------------------ */
/* 3. SPH: Wendland C4 kernel, kernel size, density, force                    */
/* ------------------------------------------------------------------------ */

/* W(r, H) = 495 / (32 pi H^3) (1 - q)^6 (1 + 6 q + 35 q^2 / 3), q = r / H < 1. */
ORC_API double orc_wendland_c4(double r, double H) {
    double q = r / H;
    if (q >= 1.0) return 0.0;
    double t = 1.0 - q;
    return 495.0 / (32.0 * M_PI * H * H * H) * pow(t, 6) * (1.0 + 6.0 * q + 35.0 / 3.0 * q * q);
}

/* dW/dr (r, H) = -1155 / (4 pi H^4) q (1 + 5 q) (1 - q)^5 for q < 1. */
ORC_API double orc_wendland_c4_dr(double r, double H) {
    double q = r / H;
    if (q >= 1.0) return 0.0;
    double t = 1.0 - q;
    return -1155.0 / (4.0 * M_PI * H * H * H * H) * q * (1.0 + 5.0 * q) * pow(t, 5);
}

/* Range query on a tree: append every particle slot within distance R of p
 * (strictly) to out; returns count.  cap bounds out; returns -1 if exceeded. */
static int64_t range_query(const orc_tree* T, const double* p, double R, int64_t* out,
                           int64_t cap) {
    int64_t cnt = 0;
    double R2 = R * R;
    for (int64_t node = 0; node < T->nn;) {
        double s = 0.0;
        for (int d = 0; d < 3; d++) {
            double t1 = T->lo[3 * node + d] - p[d];
            double t2 = p[d] - T->hi[3 * node + d];
            double t = t1 > t2 ? t1 : t2;
            if (t < 0) t = 0;
            s += t * t;
        }
        if (s >= R2) {
            node = T->next[node];
        } else if (T->leaf[node]) {
            for (int64_t j = T->nb[node]; j < T->ne[node]; j++) {
                double dx = T->xs[j] - p[0], dy = T->ys[j] - p[1], dz = T->zs[j] - p[2];
                if (dx * dx + dy * dy + dz * dz < R2) {
                    if (cnt >= cap) return -1;
                    out[cnt++] = j;
                }
            }
            node = T->next[node];
        } else {
            node++;
        }
    }
    return cnt;
}

/* N_eff(H) = (4 pi / 3) H^3 rho(H) / m_i and its derivative, over candidate
 * distances r[0..k) with masses mj[0..k) (the candidates must contain every
 * particle within H, including i itself at r = 0). */
static void neff_eval(const double* r, const double* mj, int64_t k, double mi, double H,
                      double* neff, double* dneff, double* rho) {
    double s0 = 0, s1 = 0;
    for (int64_t c = 0; c < k; c++) {
        double q = r[c] / H;
        if (q >= 1.0) continue;
        double t = 1.0 - q;
        double t5 = t * t * t * t * t;
        s0 += mj[c] * t5 * t * (1.0 + 6.0 * q + 35.0 / 3.0 * q * q);
        s1 += mj[c] * q * q * (1.0 + 5.0 * q) * t5;
    }
    /* rho = 495/(32 pi H^3) s0; N_eff = (4 pi/3) H^3 rho / m_i = (495/24) s0 / m_i;
     * dN_eff/dH = (495/24) (56/3) s1 / (m_i H). */
    *rho = 495.0 / (32.0 * M_PI * H * H * H) * s0;
    *neff = 495.0 / 24.0 * s0 / mi;
    *dneff = 495.0 / 24.0 * 56.0 / 3.0 * s1 / (mi * H);
}

/* Kernel size, density, pressure inputs for receivers idx[0..ni) (or all).
 * Root of N_eff(H) = n_ngb by Newton safeguarded with a bracket (bisection or
 * doubling when a step leaves it), until |N_eff - n_ngb| <= tol.
 * Hguess (per receiver slot, may be NULL or <= 0) seeds the iteration.
 * dlnh_out (may be NULL) receives dN_eff/dln H at the returned H.
 * Returns the number of receivers that hit max_iter. */
ORC_API int64_t orc_sph_density(int64_t n, const double* x, const double* y, const double* z,
                                const double* m, double n_ngb, double tol, int max_iter,
                                int64_t ni, const int64_t* idx, const double* Hguess,
                                double* H_out, double* rho_out, int32_t* iters_out,
                                double* dlnh_out) {
    orc_tree* T = orc_tree_build(n, x, y, z, m, NULL, 8, 64);
    int64_t* inv = malloc(n * sizeof(int64_t));
    for (int64_t s = 0; s < n; s++) inv[T->perm[s]] = s;
    int64_t nrecv = idx ? ni : n;
    int64_t nfail = 0;
#pragma omp parallel reduction(+ : nfail)
    {
        int64_t cap = 4096;
        int64_t* cand = malloc(cap * sizeof(int64_t));
        double* rr = malloc(cap * sizeof(double));
        double* mm = malloc(cap * sizeof(double));
#pragma omp for schedule(dynamic, 16)
        for (int64_t k = 0; k < nrecv; k++) {
            int64_t i = idx ? idx[k] : k;
            int64_t s = inv[i];
            double p[3] = {x[i], y[i], z[i]};
            double mi = m[i];
            double H = (Hguess && Hguess[k] > 0) ? Hguess[k] : 0.0;
            if (H <= 0) {
                /* seed from the density of the smallest node holding >= n_ngb particles */
                int64_t nd = 0;
                for (;;) {
                    int64_t best = -1;
                    if (!T->leaf[nd])
                        for (int64_t c = nd + 1; c < T->next[nd]; c = T->next[c])
                            if (T->nb[c] <= s && s < T->ne[c] && T->ne[c] - T->nb[c] >= n_ngb) best = c;
                    if (best < 0) break;
                    nd = best;
                }
                double vol = 1.0;
                for (int d = 0; d < 3; d++) {
                    double w = T->hi[3 * nd + d] - T->lo[3 * nd + d];
                    vol *= (w > 0 ? w : 1e-30);
                }
                double rho0 = T->mass[nd] / vol;
                H = cbrt(3.0 * n_ngb * mi / (4.0 * M_PI * rho0));
            }
            double Rc = 0.0;
            int64_t kc = 0;
            double lo = 0.0, hi = INFINITY;
            double neff = 0, dneff = 0, rho = 0;
            int it = 0, ok = 0;
            for (it = 1; it <= max_iter; it++) {
                if (H > Rc) {
                    Rc = 2.0 * H;
                    for (;;) {
                        kc = range_query(T, p, Rc, cand, cap);
                        if (kc >= 0) break;
                        cap *= 2;
                        cand = realloc(cand, cap * sizeof(int64_t));
                        rr = realloc(rr, cap * sizeof(double));
                        mm = realloc(mm, cap * sizeof(double));
                    }
                    for (int64_t c = 0; c < kc; c++) {
                        int64_t j = cand[c];
                        double dx = T->xs[j] - p[0], dy = T->ys[j] - p[1], dz = T->zs[j] - p[2];
                        rr[c] = sqrt(dx * dx + dy * dy + dz * dz);
                        mm[c] = T->ms[j];
                    }
                }
                neff_eval(rr, mm, kc, mi, H, &neff, &dneff, &rho);
                double f = neff - n_ngb;
                if (fabs(f) <= tol) {
                    ok = 1;
                    break;
                }
                if (f < 0) lo = H; else hi = H;
                double Hn = (dneff > 0) ? H - f / dneff : NAN;
                if (!(Hn > lo && Hn < hi)) Hn = isfinite(hi) ? 0.5 * (lo + hi) : 2.0 * H;
                H = Hn;
            }
            if (!ok) nfail++;
            H_out[k] = H;
            rho_out[k] = rho;
            if (iters_out) iters_out[k] = ok ? it : max_iter;
            if (dlnh_out) dlnh_out[k] = H * dneff; /* dN_eff / dln H at the solution */
        }
        free(cand);
        free(rr);
        free(mm);
    }
    free(inv);
    orc_tree_free(T);
    return nfail;
}

/* SPH accelerations, du/dt and signal speed for receivers idx[0..ni) (or all):
 *   dv_i/dt = -sum_j m_j [A_i gW(H_i) + A_j gW(H_j) + Pi_ij (gW(H_i) + gW(H_j))/2] r_ij
 *   du_i/dt =  sum_j m_j [A_i gW(H_i) + Pi_ij (gW(H_i) + gW(H_j))/4] v_ij . r_ij
 * with A = P / rho^2, P = (gamma - 1) rho u, c = sqrt(gamma (gamma - 1) u),
 * gW(H) r_ij = grad_i W(r_ij, H), gW(H) = -1155/(4 pi H^5) (1 + 5q)(1 - q)^5,
 * w = v_ij . r_ij / r_ij, v_sig,ij = c_i + c_j - 3 min(w, 0),
 * Pi_ij = -alpha v_sig,ij w / (rho_i + rho_j) when w < 0, else 0.
 * Pairs: every j != i with r_ij < max(H_i, H_j).  vsig_i = max over pairs
 * (c_i when i has no pair).  Velocities are the time-centred predictions.
 * H, rho, u are per particle (original order). */
ORC_API void orc_sph_force(int64_t n, const double* x, const double* y, const double* z,
                           const double* vx, const double* vy, const double* vz, const double* m,
                           const double* u, const double* H, const double* rho, double gamma,
                           double alpha, int64_t ni, const int64_t* idx, double* ax, double* ay,
                           double* az, double* dudt, double* vsig) {
    orc_tree* T = orc_tree_build(n, x, y, z, m, NULL, 8, 64);
    /* per-node maximum H for the scatter part of the search */
    double* hs = malloc(n * sizeof(double));
    for (int64_t s = 0; s < n; s++) hs[s] = H[T->perm[s]];
    for (int64_t nd = T->nn - 1; nd >= 0; nd--) {
        double h = 0;
        for (int64_t s = T->nb[nd]; s < T->ne[nd]; s++) h = hs[s] > h ? hs[s] : h;
        T->hmax[nd] = h;
    }
    int64_t nrecv = idx ? ni : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nrecv; k++) {
        int64_t i = idx ? idx[k] : k;
        double Hi = H[i], ri = rho[i];
        double Pi = (gamma - 1.0) * ri * u[i];
        double Ai = Pi / (ri * ri);
        double ci = sqrt(gamma * (gamma - 1.0) * u[i]);
        double sx = 0, sy = 0, sz = 0, su = 0, vs = ci;
        double p[3] = {x[i], y[i], z[i]};
        for (int64_t node = 0; node < T->nn;) {
            double s2 = 0.0;
            for (int d = 0; d < 3; d++) {
                double t1 = T->lo[3 * node + d] - p[d];
                double t2 = p[d] - T->hi[3 * node + d];
                double t = t1 > t2 ? t1 : t2;
                if (t < 0) t = 0;
                s2 += t * t;
            }
            double R = Hi > T->hmax[node] ? Hi : T->hmax[node];
            if (s2 >= R * R) {
                node = T->next[node];
                continue;
            }
            if (!T->leaf[node]) {
                node++;
                continue;
            }
            for (int64_t sj = T->nb[node]; sj < T->ne[node]; sj++) {
                int64_t j = T->perm[sj];
                if (j == i) continue;
                double rx = x[i] - x[j], ry = y[i] - y[j], rz = z[i] - z[j];
                double r = sqrt(rx * rx + ry * ry + rz * rz);
                double Hj = H[j];
                if (!(r < Hi || r < Hj)) continue;
                double gi = 0, gj = 0;
                if (r < Hi) {
                    double q = r / Hi;
                    gi = -1155.0 / (4.0 * M_PI * pow(Hi, 5)) * (1 + 5 * q) * pow(1 - q, 5);
                }
                if (r < Hj) {
                    double q = r / Hj;
                    gj = -1155.0 / (4.0 * M_PI * pow(Hj, 5)) * (1 + 5 * q) * pow(1 - q, 5);
                }
                double rj = rho[j];
                double Pj = (gamma - 1.0) * rj * u[j];
                double Aj = Pj / (rj * rj);
                double cj = sqrt(gamma * (gamma - 1.0) * u[j]);
                double vxij = vx[i] - vx[j], vyij = vy[i] - vy[j], vzij = vz[i] - vz[j];
                double vr = vxij * rx + vyij * ry + vzij * rz;
                double w = r > 0 ? vr / r : 0.0;
                double sig = ci + cj - 3.0 * (w < 0 ? w : 0.0);
                double Pi_ij = w < 0 ? -alpha * sig * w / (ri + rj) : 0.0;
                double gbar = 0.5 * (gi + gj);
                double f = m[j] * (Ai * gi + Aj * gj + Pi_ij * gbar);
                sx -= f * rx;
                sy -= f * ry;
                sz -= f * rz;
                su += m[j] * (Ai * gi + 0.5 * Pi_ij * gbar) * vr;
                if (sig > vs) vs = sig;
            }
            node = T->next[node];
        }
        ax[k] = sx;
        ay[k] = sy;
        az[k] = sz;
        dudt[k] = su;
        vsig[k] = vs;
    }
    free(hs);
    orc_tree_free(T);
}

/* ------------------------------------------------------------------------ */
/* 4. 3-D convolution (the U-Net of Sec. 3.3), naive loops in FP64            */
/* ------------------------------------------------------------------------ */
/* Layouts: x[b][z][y][x][c] (channels innermost); w[co][tap][ci] with
 * tap = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1) for ksize 3 (zero padding 1),
 * tap = 0 for ksize 1.
 * out[b][p][co] = bias[co] + sum_{tap, ci} in[b][p + d(tap)][ci] w[co][tap][ci] */
static int64_t vox(int b, int z, int y, int x, int S) {
    return (((int64_t)b * S + z) * S + y) * S + x;
}

ORC_API void orc_conv3d_fwd(int B, int S, int Cin, int Cout, int ksize, const double* in,
                            const double* w, const double* bias, double* out) {
    int kv = ksize == 3 ? 27 : 1, r = ksize == 3 ? 1 : 0;
#pragma omp parallel for collapse(2) schedule(static)
    for (int b = 0; b < B; b++)
        for (int z = 0; z < S; z++)
            for (int y = 0; y < S; y++)
                for (int x = 0; x < S; x++)
                    for (int co = 0; co < Cout; co++) {
                        double s = bias ? bias[co] : 0.0;
                        for (int dz = -r; dz <= r; dz++)
                            for (int dy = -r; dy <= r; dy++)
                                for (int dx = -r; dx <= r; dx++) {
                                    int Z = z + dz, Y = y + dy, X = x + dx;
                                    if (Z < 0 || Z >= S || Y < 0 || Y >= S || X < 0 || X >= S) continue;
                                    int tap = kv == 27 ? (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1) : 0;
                                    const double* ip = in + vox(b, Z, Y, X, S) * Cin;
                                    const double* wp = w + ((int64_t)co * kv + tap) * Cin;
                                    for (int ci = 0; ci < Cin; ci++) s += ip[ci] * wp[ci];
                                }
                        out[vox(b, z, y, x, S) * Cout + co] = s;
                    }
}

/* din[b][q][ci] = sum_{tap, co} dout[b][q - d(tap)][co] w[co][tap][ci] */
ORC_API void orc_conv3d_bwd_data(int B, int S, int Cin, int Cout, int ksize, const double* dout,
                                 const double* w, double* din) {
    int kv = ksize == 3 ? 27 : 1, r = ksize == 3 ? 1 : 0;
#pragma omp parallel for collapse(2) schedule(static)
    for (int b = 0; b < B; b++)
        for (int z = 0; z < S; z++)
            for (int y = 0; y < S; y++)
                for (int x = 0; x < S; x++)
                    for (int ci = 0; ci < Cin; ci++) {
                        double s = 0.0;
                        for (int dz = -r; dz <= r; dz++)
                            for (int dy = -r; dy <= r; dy++)
                                for (int dx = -r; dx <= r; dx++) {
                                    int Z = z - dz, Y = y - dy, X = x - dx;
                                    if (Z < 0 || Z >= S || Y < 0 || Y >= S || X < 0 || X >= S) continue;
                                    int tap = kv == 27 ? (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1) : 0;
                                    const double* gp = dout + vox(b, Z, Y, X, S) * Cout;
                                    for (int co = 0; co < Cout; co++)
                                        s += gp[co] * w[((int64_t)co * kv + tap) * Cin + ci];
                                }
                        din[vox(b, z, y, x, S) * Cin + ci] = s;
                    }
}

/* dw[co][tap][ci] = sum_{b, p} dout[b][p][co] in[b][p + d(tap)][ci]; db[co] = sum dout */
ORC_API void orc_conv3d_bwd_weight(int B, int S, int Cin, int Cout, int ksize, const double* in,
                                   const double* dout, double* dw, double* db) {
    int kv = ksize == 3 ? 27 : 1, r = ksize == 3 ? 1 : 0;
#pragma omp parallel for schedule(static)
    for (int co = 0; co < Cout; co++) {
        for (int t = 0; t < kv * Cin; t++) dw[(int64_t)co * kv * Cin + t] = 0.0;
        double sb = 0.0;
        for (int b = 0; b < B; b++)
            for (int z = 0; z < S; z++)
                for (int y = 0; y < S; y++)
                    for (int x = 0; x < S; x++) {
                        double g = dout[vox(b, z, y, x, S) * Cout + co];
                        sb += g;
                        for (int dz = -r; dz <= r; dz++)
                            for (int dy = -r; dy <= r; dy++)
                                for (int dx = -r; dx <= r; dx++) {
                                    int Z = z + dz, Y = y + dy, X = x + dx;
                                    if (Z < 0 || Z >= S || Y < 0 || Y >= S || X < 0 || X >= S) continue;
                                    int tap = kv == 27 ? (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1) : 0;
                                    const double* ip = in + vox(b, Z, Y, X, S) * Cin;
                                    double* wp = dw + ((int64_t)co * kv + tap) * Cin;
                                    for (int ci = 0; ci < Cin; ci++) wp[ci] += g * ip[ci];
                                }
                    }
        if (db) db[co] = sb;
    }
}

/* ------------------------------------------------------------------------ */
/* 5. Particle-to-voxel mapping (Sec. 3.3): SPH kernel convolution for the    */
/*    density, Shepard-normalised kernel averages for T and velocity          */
/* ------------------------------------------------------------------------ */
/* Voxel centres c - side/2 + (i + 1/2) side/grid; out[v][5] = log10 rho
 * (floored at rho_floor), log10 T (floored at t_floor), vx, vy, vz; voxels
 * with no kernel overlap take amb[0..4]. */
ORC_API void orc_voxelize(int64_t n, const double* x, const double* y, const double* z,
                          const double* m, const double* H, const double* T, const double* vx,
                          const double* vy, const double* vz, const double* center, double side,
                          int grid, const double* amb, double rho_floor, double t_floor,
                          double* out) {
    double dv = side / grid;
    int64_t nv = (int64_t)grid * grid * grid;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t v = 0; v < nv; v++) {
        int X = (int)(v % grid), Y = (int)((v / grid) % grid), Z = (int)(v / ((int64_t)grid * grid));
        double px = center[0] - side / 2 + (X + 0.5) * dv;
        double py = center[1] - side / 2 + (Y + 0.5) * dv;
        double pz = center[2] - side / 2 + (Z + 0.5) * dv;
        double sr = 0, sw = 0, st = 0, s1 = 0, s2 = 0, s3 = 0;
        for (int64_t j = 0; j < n; j++) {
            double dx = px - x[j], dy = py - y[j], dz = pz - z[j];
            if (fabs(dx) >= H[j] || fabs(dy) >= H[j] || fabs(dz) >= H[j]) continue;
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double w = orc_wendland_c4(r, H[j]);
            sr += m[j] * w;
            sw += w;
            st += w * T[j];
            s1 += w * vx[j];
            s2 += w * vy[j];
            s3 += w * vz[j];
        }
        double* o = out + v * 5;
        o[0] = log10(sr > rho_floor ? sr : rho_floor);
        if (sw > 0) {
            double t = st / sw;
            o[1] = log10(t > t_floor ? t : t_floor);
            o[2] = s1 / sw;
            o[3] = s2 / sw;
            o[4] = s3 / sw;
        } else {
            for (int q = 1; q < 5; q++) o[q] = amb[q];
        }
    }
}
