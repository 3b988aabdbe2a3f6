/*
 * FP64 CPU oracle for exact mesh-to-mesh minimum / maximum distance.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Plain, slow, double precision.
 *
 * Definitions followed:
 *   - D_min / D_max between two point sets (gDist Sec. 3, Eqs. 1-2), Euclidean.
 *   - Conventional AABB bounds d_min^L, d_max^U (Sec. 4, the f_min / f_max
 *     per-axis formulas) and the enhanced bounds d_min^U / d_max^L evaluated
 *     literally over the 36 pairs of box face rectangles (Sec. 4).
 *   - Penetration gives distance zero (Sec. 7).
 * The exact triangle-triangle distance is the plain geometric definition
 * written out (the paper names a narrow phase but gives no routine):
 *   the distance between two closed triangles is attained either at a vertex
 *   of one against the other triangle, or between two edges; if neither
 *   feature pair gives zero but an edge of one triangle crosses the other
 *   triangle, the triangles intersect and the distance is zero.
 * The maximum over two triangles is attained at a vertex pair (the norm is
 * convex, so its maximum over a product of polytopes sits at vertices).
 */
#define _GNU_SOURCE
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* small vector helpers                                                */
/* ------------------------------------------------------------------ */
static void vsub(const double* a, const double* b, double* o) {
  o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2];
}
static double vdot(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void vcross(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
static void vaxpy(const double* a, double s, const double* d, double* o) {
  o[0] = a[0] + s * d[0]; o[1] = a[1] + s * d[1]; o[2] = a[2] + s * d[2];
}
static void vcopy(const double* a, double* o) { o[0] = a[0]; o[1] = a[1]; o[2] = a[2]; }
static double vdist(const double* a, const double* b) {
  double d[3]; vsub(a, b, d); return sqrt(vdot(d, d));
}

void orc_pose_points(const float* v, int64_t n, const double pose[12], double* out) {
  for (int64_t i = 0; i < n; ++i) {
    double x = (double)v[3 * i + 0], y = (double)v[3 * i + 1], z = (double)v[3 * i + 2];
    for (int r = 0; r < 3; ++r)
      out[3 * i + r] = ((pose[3 * r + 0] * x + pose[3 * r + 1] * y) + pose[3 * r + 2] * z) + pose[9 + r];
  }
}

/* ------------------------------------------------------------------ */
/* point / segment / triangle primitives                               */
/* ------------------------------------------------------------------ */
double orc_point_segment(const double p[3], const double a[3], const double b[3], double q[3]) {
  double ab[3], ap[3];
  vsub(b, a, ab);
  vsub(p, a, ap);
  double L = vdot(ab, ab), t = 0.0;
  if (L > 0.0) {
    t = vdot(ap, ab) / L;
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
  }
  double c[3];
  vaxpy(a, t, ab, c);
  if (q) vcopy(c, q);
  return vdist(p, c);
}

/* 1 if x (assumed in the plane of a,b,c with normal n) lies in the closed triangle. */
static int inside_closed(const double* x, const double* a, const double* b, const double* c,
                         const double* n) {
  double e[3], w[3], k[3];
  vsub(b, a, e); vsub(x, a, w); vcross(e, w, k);
  if (vdot(k, n) < 0.0) return 0;
  vsub(c, b, e); vsub(x, b, w); vcross(e, w, k);
  if (vdot(k, n) < 0.0) return 0;
  vsub(a, c, e); vsub(x, c, w); vcross(e, w, k);
  if (vdot(k, n) < 0.0) return 0;
  return 1;
}

double orc_point_triangle(const double p[3], const double t[9], double q[3]) {
  const double *a = t, *b = t + 3, *c = t + 6;
  double ab[3], ac[3], n[3];
  vsub(b, a, ab); vsub(c, a, ac); vcross(ab, ac, n);
  double nn = vdot(n, n);
  if (nn > 0.0) {
    double ap[3], x[3];
    vsub(p, a, ap);
    double s = vdot(ap, n) / nn;
    vaxpy(p, -s, n, x);            /* projection onto the plane */
    if (inside_closed(x, a, b, c, n)) {
      if (q) vcopy(x, q);
      return vdist(p, x);
    }
  }
  /* outside (or degenerate): nearest of the three closed edges */
  double best = INFINITY, tmp[3], bq[3] = {0, 0, 0};
  const double* v[3] = {a, b, c};
  for (int i = 0; i < 3; ++i) {
    double d = orc_point_segment(p, v[i], v[(i + 1) % 3], tmp);
    if (d < best) { best = d; vcopy(tmp, bq); }
  }
  if (q) vcopy(bq, q);
  return best;
}

double orc_segment_segment(const double p0[3], const double p1[3], const double q0[3],
                           const double q1[3], double cp[3], double cq[3]) {
  /* |p0 + s d1 - q0 - t d2|^2 is a convex quadratic on [0,1]^2: its minimum is
   * the interior stationary point (when it exists and lies inside) or a point
   * on one of the four sides, each side being an endpoint-to-segment problem. */
  double best = INFINITY, bp[3] = {0, 0, 0}, bq[3] = {0, 0, 0}, tmp[3], d;
  d = orc_point_segment(p0, q0, q1, tmp);
  if (d < best) { best = d; vcopy(p0, bp); vcopy(tmp, bq); }
  d = orc_point_segment(p1, q0, q1, tmp);
  if (d < best) { best = d; vcopy(p1, bp); vcopy(tmp, bq); }
  d = orc_point_segment(q0, p0, p1, tmp);
  if (d < best) { best = d; vcopy(tmp, bp); vcopy(q0, bq); }
  d = orc_point_segment(q1, p0, p1, tmp);
  if (d < best) { best = d; vcopy(tmp, bp); vcopy(q1, bq); }
  double d1[3], d2[3], r[3];
  vsub(p1, p0, d1); vsub(q1, q0, d2); vsub(p0, q0, r);
  double a = vdot(d1, d1), e = vdot(d2, d2), b = vdot(d1, d2);
  double c = vdot(d1, r), f = vdot(d2, r);
  double den = a * e - b * b;
  if (den > 0.0) {
    double s = (b * f - c * e) / den;
    double t = (a * f - b * c) / den;
    if (s >= 0.0 && s <= 1.0 && t >= 0.0 && t <= 1.0) {
      double X[3], Y[3];
      vaxpy(p0, s, d1, X);
      vaxpy(q0, t, d2, Y);
      d = vdist(X, Y);
      if (d < best) { best = d; vcopy(X, bp); vcopy(Y, bq); }
    }
  }
  if (cp) vcopy(bp, cp);
  if (cq) vcopy(bq, cq);
  return best;
}

int orc_segment_pierces(const double p0[3], const double p1[3], const double t[9], double x[3]) {
  const double *a = t, *b = t + 3, *c = t + 6;
  double ab[3], ac[3], n[3], w[3];
  vsub(b, a, ab); vsub(c, a, ac); vcross(ab, ac, n);
  if (vdot(n, n) == 0.0) return 0;
  vsub(p0, a, w);
  double s0 = vdot(w, n);
  vsub(p1, a, w);
  double s1 = vdot(w, n);
  if ((s0 > 0.0 && s1 > 0.0) || (s0 < 0.0 && s1 < 0.0)) return 0;
  if (s0 == s1) return 0;          /* segment lies in the plane: not a single crossing */
  double lam = s0 / (s0 - s1), d[3], X[3];
  vsub(p1, p0, d);
  vaxpy(p0, lam, d, X);
  if (!inside_closed(X, a, b, c, n)) return 0;
  if (x) vcopy(X, x);
  return 1;
}

double orc_tri_tri_min(const double P[9], const double Q[9], double cp[3], double cq[3]) {
  double best = INFINITY, bp[3] = {0, 0, 0}, bq[3] = {0, 0, 0}, t1[3], t2[3], d;
  /* vertices of P against Q, then vertices of Q against P */
  for (int i = 0; i < 3; ++i) {
    d = orc_point_triangle(P + 3 * i, Q, t1);
    if (d < best) { best = d; vcopy(P + 3 * i, bp); vcopy(t1, bq); }
  }
  for (int j = 0; j < 3; ++j) {
    d = orc_point_triangle(Q + 3 * j, P, t1);
    if (d < best) { best = d; vcopy(t1, bp); vcopy(Q + 3 * j, bq); }
  }
  /* the nine edge pairs */
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      d = orc_segment_segment(P + 3 * i, P + 3 * ((i + 1) % 3), Q + 3 * j, Q + 3 * ((j + 1) % 3), t1, t2);
      if (d < best) { best = d; vcopy(t1, bp); vcopy(t2, bq); }
    }
  /* an edge crossing the interior of the other triangle means they intersect */
  if (best > 0.0) {
    for (int i = 0; i < 3; ++i)
      if (orc_segment_pierces(P + 3 * i, P + 3 * ((i + 1) % 3), Q, t1)) {
        best = 0.0; vcopy(t1, bp); vcopy(t1, bq); goto done;
      }
    for (int j = 0; j < 3; ++j)
      if (orc_segment_pierces(Q + 3 * j, Q + 3 * ((j + 1) % 3), P, t1)) {
        best = 0.0; vcopy(t1, bp); vcopy(t1, bq); goto done;
      }
  }
done:
  if (cp) vcopy(bp, cp);
  if (cq) vcopy(bq, cq);
  return best;
}

double orc_tri_tri_max(const double P[9], const double Q[9], double cp[3], double cq[3]) {
  double best = -1.0;
  int bi = 0, bj = 0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double d = vdist(P + 3 * i, Q + 3 * j);
      if (d > best) { best = d; bi = i; bj = j; }
    }
  if (cp) vcopy(P + 3 * bi, cp);
  if (cq) vcopy(Q + 3 * bj, cq);
  return best;
}

/* ------------------------------------------------------------------ */
/* AABB distance bounds, literally as the paper states them            */
/* ------------------------------------------------------------------ */
/* f_max of Sec. 4 over the three axes: largest distance between two (possibly
 * flat) axis-aligned boxes, squared. */
static double box_far2(const double* lo1, const double* hi1, const double* lo2, const double* hi2) {
  double s = 0.0;
  for (int i = 0; i < 3; ++i) {
    double u = fabs(lo1[i] - hi2[i]), v = fabs(hi1[i] - lo2[i]);
    double f = u > v ? u : v;
    s += f * f;
  }
  return s;
}
/* f_min of Sec. 4 over the three axes: smallest distance, squared. */
static double box_near2(const double* lo1, const double* hi1, const double* lo2, const double* hi2) {
  double s = 0.0;
  for (int i = 0; i < 3; ++i) {
    int overlap = (lo1[i] <= hi2[i]) && (lo2[i] <= hi1[i]);
    double f = 0.0;
    if (!overlap) {
      double u = fabs(lo1[i] - hi2[i]), v = fabs(hi1[i] - lo2[i]);
      f = u < v ? u : v;
    }
    s += f * f;
  }
  return s;
}
/* face k of box (lo,hi): axis k%3, side k/3 (0 = min face, 1 = max face) */
static void box_face(const double* lo, const double* hi, int k, double* flo, double* fhi) {
  vcopy(lo, flo); vcopy(hi, fhi);
  int ax = k % 3;
  double v = (k / 3) ? hi[ax] : lo[ax];
  flo[ax] = v; fhi[ax] = v;
}

void orc_box_bounds(const double a[6], const double b[6], double out[4]) {
  const double *alo = a, *ahi = a + 3, *blo = b, *bhi = b + 3;
  out[0] = sqrt(box_near2(alo, ahi, blo, bhi));
  out[2] = sqrt(box_far2(alo, ahi, blo, bhi));
  double up = INFINITY, lo = -INFINITY;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      double fal[3], fah[3], fbl[3], fbh[3];
      box_face(alo, ahi, i, fal, fah);
      box_face(blo, bhi, j, fbl, fbh);
      double m = box_far2(fal, fah, fbl, fbh);   /* farthest points of the two faces */
      double n = box_near2(fal, fah, fbl, fbh);  /* nearest points of the two faces  */
      if (m < up) up = m;
      if (n > lo) lo = n;
    }
  out[1] = sqrt(up);
  out[3] = sqrt(lo);
}

/* ------------------------------------------------------------------ */
/* mesh helpers                                                        */
/* ------------------------------------------------------------------ */
typedef struct {
  const double* v;     /* posed vertices, 3 per vertex */
  const uint32_t* f;   /* triangles */
  int64_t nf;
} pmesh;

static void tri_coords(const pmesh* m, int64_t t, double* out9) {
  for (int k = 0; k < 3; ++k) vcopy(m->v + 3 * (int64_t)m->f[3 * t + k], out9 + 3 * k);
}

static int check_mesh(const float* v, int64_t nv, const uint32_t* f, int64_t nf) {
  if (!v || !f || nv <= 0 || nf <= 0) return 1;
  for (int64_t i = 0; i < 3 * nf; ++i)
    if ((int64_t)f[i] >= nv) return 2;
  for (int64_t i = 0; i < 3 * nv; ++i)
    if (!isfinite(v[i])) return 3;
  return 0;
}

static double pair_dist(const pmesh* A, const pmesh* B, int64_t a, int64_t b, int mode,
                        double* cp, double* cq) {
  double P[9], Q[9];
  tri_coords(A, a, P);
  tri_coords(B, b, Q);
  return mode ? orc_tri_tri_max(P, Q, cp, cq) : orc_tri_tri_min(P, Q, cp, cq);
}

/* tie list: dynamic array of (a, b, d) */
typedef struct {
  int64_t* ab;
  double* d;
  int64_t n, cap;
} tlist;

static void tl_push(tlist* t, int64_t a, int64_t b, double d) {
  if (t->n == t->cap) {
    t->cap = t->cap ? 2 * t->cap : 256;
    t->ab = (int64_t*)realloc(t->ab, sizeof(int64_t) * 2 * t->cap);
    t->d = (double*)realloc(t->d, sizeof(double) * t->cap);
  }
  t->ab[2 * t->n] = a;
  t->ab[2 * t->n + 1] = b;
  t->d[t->n] = d;
  t->n++;
}
static void tl_free(tlist* t) { free(t->ab); free(t->d); memset(t, 0, sizeof(*t)); }

static int cmp_pair(const void* x, const void* y) {
  const int64_t* p = (const int64_t*)x;
  const int64_t* q = (const int64_t*)y;
  if (p[0] != q[0]) return p[0] < q[0] ? -1 : 1;
  if (p[1] != q[1]) return p[1] < q[1] ? -1 : 1;
  return 0;
}

/* keep the entries of t within tau of D (min mode: d <= D+tau, max: d >= D-tau),
 * sort them lexicographically, fill out / ties. */
static void finish_result(tlist* t, double D, double tau, int mode, const pmesh* A, const pmesh* B,
                          orc_result_t* out, int64_t* ties, int64_t tie_cap) {
  int64_t m = 0;
  for (int64_t i = 0; i < t->n; ++i) {
    int keep = mode ? (t->d[i] >= D - tau) : (t->d[i] <= D + tau);
    if (keep) {
      t->ab[2 * m] = t->ab[2 * i];
      t->ab[2 * m + 1] = t->ab[2 * i + 1];
      t->d[m] = t->d[i];
      ++m;
    }
  }
  t->n = m;
  qsort(t->ab, (size_t)m, 2 * sizeof(int64_t), cmp_pair);
  out->distance = D;
  out->n_ties = m;
  if (ties)
    for (int64_t i = 0; i < m && i < tie_cap; ++i) {
      ties[2 * i] = t->ab[2 * i];
      ties[2 * i + 1] = t->ab[2 * i + 1];
    }
  if (m > 0) {
    out->tri_a = t->ab[0];
    out->tri_b = t->ab[1];
    out->pair_distance = pair_dist(A, B, out->tri_a, out->tri_b, mode, out->point_a, out->point_b);
  } else {
    out->tri_a = out->tri_b = -1;
  }
}

/* ------------------------------------------------------------------ */
/* brute force                                                         */
/* ------------------------------------------------------------------ */
typedef struct {
  const pmesh *A, *B;
  int mode;
  int pass;            /* 1: extreme value, 2: collect ties */
  double D, tau;
  int64_t* next;       /* shared row counter */
  double local;        /* pass 1 result */
  tlist ties;          /* pass 2 result */
  int64_t tested;
} bf_job;

static void* bf_worker(void* arg) {
  bf_job* j = (bf_job*)arg;
  double loc = j->mode ? -1.0 : INFINITY;
  const int64_t chunk = 16;
  for (;;) {
    int64_t a0 = __sync_fetch_and_add(j->next, chunk);
    if (a0 >= j->A->nf) break;
    int64_t a1 = a0 + chunk < j->A->nf ? a0 + chunk : j->A->nf;
    for (int64_t a = a0; a < a1; ++a)
      for (int64_t b = 0; b < j->B->nf; ++b) {
        double d = pair_dist(j->A, j->B, a, b, j->mode, NULL, NULL);
        j->tested++;
        if (j->pass == 1) {
          if (j->mode ? (d > loc) : (d < loc)) loc = d;
        } else {
          int keep = j->mode ? (d >= j->D - j->tau) : (d <= j->D + j->tau);
          if (keep) tl_push(&j->ties, a, b, d);
        }
      }
  }
  j->local = loc;
  return NULL;
}

static double* pose_all(const float* v, int64_t nv, const double pose[12]) {
  double* out = (double*)malloc(sizeof(double) * 3 * (size_t)nv);
  orc_pose_points(v, nv, pose, out);
  return out;
}

int orc_brute(const float* va, int64_t nva, const uint32_t* fa, int64_t nfa, const double pose_a[12],
              const float* vb, int64_t nvb, const uint32_t* fb, int64_t nfb, const double pose_b[12],
              int mode, double tau, int threads, orc_result_t* out, int64_t* ties, int64_t tie_cap) {
  if (check_mesh(va, nva, fa, nfa) || check_mesh(vb, nvb, fb, nfb) || !out) return 1;
  if (mode != 0 && mode != 1) return 1;
  if (threads < 1) threads = 1;
  memset(out, 0, sizeof(*out));
  double* pa = pose_all(va, nva, pose_a);
  double* pb = pose_all(vb, nvb, pose_b);
  pmesh A = {pa, fa, nfa}, B = {pb, fb, nfb};
  bf_job* jobs = (bf_job*)calloc((size_t)threads, sizeof(bf_job));
  pthread_t* th = (pthread_t*)calloc((size_t)threads, sizeof(pthread_t));
  double D = mode ? -1.0 : INFINITY;
  int64_t tested = 0;
  for (int pass = 1; pass <= 2; ++pass) {
    int64_t next = 0;
    for (int i = 0; i < threads; ++i) {
      jobs[i].A = &A; jobs[i].B = &B; jobs[i].mode = mode; jobs[i].pass = pass;
      jobs[i].D = D; jobs[i].tau = tau; jobs[i].next = &next;
      pthread_create(&th[i], NULL, bf_worker, &jobs[i]);
    }
    for (int i = 0; i < threads; ++i) pthread_join(th[i], NULL);
    if (pass == 1)
      for (int i = 0; i < threads; ++i) {
        if (mode ? (jobs[i].local > D) : (jobs[i].local < D)) D = jobs[i].local;
        tested += jobs[i].tested;
        jobs[i].tested = 0;
      }
  }
  tlist all = {0};
  for (int i = 0; i < threads; ++i) {
    for (int64_t k = 0; k < jobs[i].ties.n; ++k)
      tl_push(&all, jobs[i].ties.ab[2 * k], jobs[i].ties.ab[2 * k + 1], jobs[i].ties.d[k]);
    tl_free(&jobs[i].ties);
  }
  finish_result(&all, D, tau, mode, &A, &B, out, ties, tie_cap);
  out->pairs_tested = tested;
  tl_free(&all);
  free(jobs); free(th); free(pa); free(pb);
  return 0;
}

/* ------------------------------------------------------------------ */
/* the oracle's own BVH: top-down median split, at most 4 triangles     */
/* per leaf, searched best-first                                        */
/* ------------------------------------------------------------------ */
typedef struct {
  double lo[3], hi[3];
  int64_t left, right;   /* children (-1 for a leaf) */
  int64_t start, count;  /* triangle range in the permutation (leaves) */
} onode;

typedef struct {
  onode* n;
  int64_t nn, cap;
  int64_t* perm;         /* triangle ids */
  double* cen;           /* centroids, 3 per triangle */
  const pmesh* m;
} otree;

static int64_t ot_new(otree* t) {
  if (t->nn == t->cap) {
    t->cap = t->cap ? 2 * t->cap : 1024;
    t->n = (onode*)realloc(t->n, sizeof(onode) * (size_t)t->cap);
  }
  return t->nn++;
}

/* three-way quickselect: reorder perm[lo,hi) so that perm[k] holds the element
 * of rank k by centroid coordinate ax, smaller ones before, larger after. */
static void select_kth(int64_t* perm, const double* cen, int ax, int64_t lo, int64_t hi, int64_t k) {
  while (hi - lo > 1) {
    double a = cen[3 * perm[lo] + ax], b = cen[3 * perm[(lo + hi) / 2] + ax], c = cen[3 * perm[hi - 1] + ax];
    double piv = (a < b) ? ((b < c) ? b : (a < c ? c : a)) : ((a < c) ? a : (b < c ? c : b));
    int64_t lt = lo, i = lo, gt = hi;
    while (i < gt) {
      double x = cen[3 * perm[i] + ax];
      if (x < piv) { int64_t s = perm[lt]; perm[lt] = perm[i]; perm[i] = s; ++lt; ++i; }
      else if (x > piv) { --gt; int64_t s = perm[gt]; perm[gt] = perm[i]; perm[i] = s; }
      else ++i;
    }
    if (k < lt) hi = lt;
    else if (k >= gt) lo = gt;
    else return;
  }
}

static int64_t ot_build(otree* t, int64_t start, int64_t count) {
  int64_t id = ot_new(t);
  onode nd;
  for (int k = 0; k < 3; ++k) { nd.lo[k] = INFINITY; nd.hi[k] = -INFINITY; }
  double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = start; i < start + count; ++i) {
    int64_t tri = t->perm[i];
    for (int c = 0; c < 3; ++c) {
      const double* p = t->m->v + 3 * (int64_t)t->m->f[3 * tri + c];
      for (int k = 0; k < 3; ++k) {
        if (p[k] < nd.lo[k]) nd.lo[k] = p[k];
        if (p[k] > nd.hi[k]) nd.hi[k] = p[k];
      }
    }
    for (int k = 0; k < 3; ++k) {
      double x = t->cen[3 * tri + k];
      if (x < clo[k]) clo[k] = x;
      if (x > chi[k]) chi[k] = x;
    }
  }
  nd.start = start;
  nd.count = count;
  nd.left = nd.right = -1;
  if (count > 4) {
    int ax = 0;
    for (int k = 1; k < 3; ++k)
      if (chi[k] - clo[k] > chi[ax] - clo[ax]) ax = k;
    int64_t half = count / 2;
    select_kth(t->perm, t->cen, ax, start, start + count, start + half);
    int64_t l = ot_build(t, start, half);
    int64_t r = ot_build(t, start + half, count - half);
    nd.left = l;
    nd.right = r;
  }
  t->n[id] = nd;
  return id;
}

static void ot_init(otree* t, const pmesh* m) {
  memset(t, 0, sizeof(*t));
  t->m = m;
  t->perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)m->nf);
  t->cen = (double*)malloc(sizeof(double) * 3 * (size_t)m->nf);
  for (int64_t i = 0; i < m->nf; ++i) {
    t->perm[i] = i;
    for (int k = 0; k < 3; ++k) {
      double s = 0.0;
      for (int c = 0; c < 3; ++c) s += m->v[3 * (int64_t)m->f[3 * i + c] + k];
      t->cen[3 * i + k] = s / 3.0;
    }
  }
  ot_build(t, 0, m->nf);
}
static void ot_free(otree* t) { free(t->n); free(t->perm); free(t->cen); }

/* binary min-heap of (key, node a, node b) */
typedef struct { double key; int64_t a, b; } hent;
typedef struct { hent* h; int64_t n, cap; } heap;

static void hp_push(heap* q, double key, int64_t a, int64_t b) {
  if (q->n == q->cap) {
    q->cap = q->cap ? 2 * q->cap : 1024;
    q->h = (hent*)realloc(q->h, sizeof(hent) * (size_t)q->cap);
  }
  int64_t i = q->n++;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (q->h[p].key <= key) break;
    q->h[i] = q->h[p];
    i = p;
  }
  q->h[i].key = key; q->h[i].a = a; q->h[i].b = b;
}
static hent hp_pop(heap* q) {
  hent top = q->h[0];
  hent last = q->h[--q->n];
  int64_t i = 0;
  for (;;) {
    int64_t l = 2 * i + 1, r = l + 1, s = i;
    double ks = last.key;
    if (l < q->n && q->h[l].key < ks) { s = l; ks = q->h[l].key; }
    if (r < q->n && q->h[r].key < ks) { s = r; }
    if (s == i) break;
    q->h[i] = q->h[s];
    i = s;
  }
  if (q->n > 0) q->h[i] = last;
  return top;
}

/* conventional bounds between two oracle nodes (Sec. 4): lower bound of the
 * min distance, and upper bound of the max distance */
static double node_lower(const onode* x, const onode* y) { return sqrt(box_near2(x->lo, x->hi, y->lo, y->hi)); }
static double node_upper(const onode* x, const onode* y) { return sqrt(box_far2(x->lo, x->hi, y->lo, y->hi)); }

static double node_diag2(const onode* x) {
  double s = 0.0;
  for (int k = 0; k < 3; ++k) s += (x->hi[k] - x->lo[k]) * (x->hi[k] - x->lo[k]);
  return s;
}

int orc_bvh(const float* va, int64_t nva, const uint32_t* fa, int64_t nfa, const double pose_a[12],
            const float* vb, int64_t nvb, const uint32_t* fb, int64_t nfb, const double pose_b[12],
            int mode, double tau, orc_result_t* out, int64_t* ties, int64_t tie_cap) {
  if (check_mesh(va, nva, fa, nfa) || check_mesh(vb, nvb, fb, nfb) || !out) return 1;
  if (mode != 0 && mode != 1) return 1;
  memset(out, 0, sizeof(*out));
  double* pa = pose_all(va, nva, pose_a);
  double* pb = pose_all(vb, nvb, pose_b);
  pmesh A = {pa, fa, nfa}, B = {pb, fb, nfb};
  otree TA, TB;
  ot_init(&TA, &A);
  ot_init(&TB, &B);
  heap q = {0};
  tlist tl = {0};
  double best = mode ? -1.0 : INFINITY;
  int64_t tested = 0;
  /* min mode: key = lower bound, expand smallest first; max mode: key = -upper */
#define KEY(x, y) (mode ? -node_upper((x), (y)) : node_lower((x), (y)))
#define PRUNED(k) (mode ? (-(k) < best - tau) : ((k) > best + tau))
  hp_push(&q, KEY(&TA.n[0], &TB.n[0]), 0, 0);
  while (q.n > 0) {
    hent e = hp_pop(&q);
    if (PRUNED(e.key)) break;    /* every remaining entry is at least as bad */
    const onode* x = &TA.n[e.a];
    const onode* y = &TB.n[e.b];
    if (x->left < 0 && y->left < 0) {
      for (int64_t i = x->start; i < x->start + x->count; ++i)
        for (int64_t j = y->start; j < y->start + y->count; ++j) {
          int64_t ta = TA.perm[i], tb = TB.perm[j];
          double d = pair_dist(&A, &B, ta, tb, mode, NULL, NULL);
          ++tested;
          if (mode ? (d > best) : (d < best)) best = d;
          if (mode ? (d >= best - tau) : (d <= best + tau)) tl_push(&tl, ta, tb, d);
        }
      continue;
    }
    int split_a;
    if (x->left < 0) split_a = 0;
    else if (y->left < 0) split_a = 1;
    else split_a = node_diag2(x) >= node_diag2(y);
    if (split_a) {
      int64_t c[2] = {x->left, x->right};
      for (int k = 0; k < 2; ++k) {
        double key = KEY(&TA.n[c[k]], y);
        if (!PRUNED(key)) hp_push(&q, key, c[k], e.b);
      }
    } else {
      int64_t c[2] = {y->left, y->right};
      for (int k = 0; k < 2; ++k) {
        double key = KEY(x, &TB.n[c[k]]);
        if (!PRUNED(key)) hp_push(&q, key, e.a, c[k]);
      }
    }
  }
#undef KEY
#undef PRUNED
  finish_result(&tl, best, tau, mode, &A, &B, out, ties, tie_cap);
  out->pairs_tested = tested;
  tl_free(&tl);
  free(q.h);
  ot_free(&TA);
  ot_free(&TB);
  free(pa);
  free(pb);
  return 0;
}

/* ------------------------------------------------------------------ */
/* D_max over vertex pairs                                             */
/* ------------------------------------------------------------------ */
typedef struct {
  const double *pa, *pb;
  int64_t na, nb;
  int64_t* next;
  double best;
} vp_job;

static void* vp_worker(void* arg) {
  vp_job* j = (vp_job*)arg;
  double best = -1.0;
  for (;;) {
    int64_t a0 = __sync_fetch_and_add(j->next, 64);
    if (a0 >= j->na) break;
    int64_t a1 = a0 + 64 < j->na ? a0 + 64 : j->na;
    /* squared distances compare like distances; one square root at the end */
    for (int64_t a = a0; a < a1; ++a)
      for (int64_t b = 0; b < j->nb; ++b) {
        double e[3];
        vsub(j->pa + 3 * a, j->pb + 3 * b, e);
        double d2 = vdot(e, e);
        if (d2 > best) best = d2;
      }
  }
  j->best = best < 0.0 ? best : sqrt(best);
  return NULL;
}

double orc_max_vertex_pairs(const float* va, int64_t nva, const double pose_a[12],
                            const float* vb, int64_t nvb, const double pose_b[12], int threads) {
  if (threads < 1) threads = 1;
  double* pa = pose_all(va, nva, pose_a);
  double* pb = pose_all(vb, nvb, pose_b);
  vp_job* jobs = (vp_job*)calloc((size_t)threads, sizeof(vp_job));
  pthread_t* th = (pthread_t*)calloc((size_t)threads, sizeof(pthread_t));
  int64_t next = 0;
  for (int i = 0; i < threads; ++i) {
    jobs[i].pa = pa; jobs[i].pb = pb; jobs[i].na = nva; jobs[i].nb = nvb; jobs[i].next = &next;
    pthread_create(&th[i], NULL, vp_worker, &jobs[i]);
  }
  double best = -1.0;
  for (int i = 0; i < threads; ++i) {
    pthread_join(th[i], NULL);
    if (jobs[i].best > best) best = jobs[i].best;
  }
  free(jobs); free(th); free(pa); free(pb);
  return best;
}

/* ------------------------------------------------------------------ */
/* per-vertex farthest distance (rows of the vertex-pair maximum)      */
/* ------------------------------------------------------------------ */
typedef struct {
  const double *pa, *pb;
  int64_t na, nb;
  int64_t* next;
  double* rowmax;
} rm_job;

static void* rm_worker(void* arg) {
  rm_job* j = (rm_job*)arg;
  for (;;) {
    int64_t a0 = __sync_fetch_and_add(j->next, 64);
    if (a0 >= j->na) break;
    int64_t a1 = a0 + 64 < j->na ? a0 + 64 : j->na;
    for (int64_t a = a0; a < a1; ++a) {
      double best = -1.0;
      for (int64_t b = 0; b < j->nb; ++b) {
        double e[3];
        vsub(j->pa + 3 * a, j->pb + 3 * b, e);
        double d2 = vdot(e, e);
        if (d2 > best) best = d2;
      }
      j->rowmax[a] = sqrt(best);
    }
  }
  return NULL;
}

void orc_vertex_row_max(const float* va, int64_t nva, const double pose_a[12],
                        const float* vb, int64_t nvb, const double pose_b[12], int threads, double* rowmax) {
  if (threads < 1) threads = 1;
  double* pa = pose_all(va, nva, pose_a);
  double* pb = pose_all(vb, nvb, pose_b);
  rm_job* jobs = (rm_job*)calloc((size_t)threads, sizeof(rm_job));
  pthread_t* th = (pthread_t*)calloc((size_t)threads, sizeof(pthread_t));
  int64_t next = 0;
  for (int i = 0; i < threads; ++i) {
    jobs[i].pa = pa; jobs[i].pb = pb; jobs[i].na = nva; jobs[i].nb = nvb; jobs[i].next = &next;
    jobs[i].rowmax = rowmax;
    pthread_create(&th[i], NULL, rm_worker, &jobs[i]);
  }
  for (int i = 0; i < threads; ++i) pthread_join(th[i], NULL);
  free(jobs); free(th); free(pa); free(pb);
}
