/*
 * FP64 CPU oracle for exact mesh-to-mesh minimum / maximum distance.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or constant with the GPU library: it is a plain, slow restatement
 * of the definitions in the gDist paper (Fan et al., SIGGRAPH Asia 2024):
 *
 *   D_min = min over p in P, q in Q of |p - q|,
 *   D_max = max over p in P, q in Q of |p - q|      (Sec. 3, Eqs. 1-2)
 *
 * where P and Q are the two posed triangle meshes (closed triangles) and the
 * norm is Euclidean.  Everything is computed in double precision with
 * round-to-nearest and no contraction (built with -ffp-contract=off).
 *
 * Poses are 12 doubles: R row-major (3x3) then t; world = R x + t.
 * Vertices are float32 triples, triangles uint32 triples (0-based).
 *
 * Pins: every routine here is checked by the CPU test suite against closed
 * forms, brute-force sampling and hand cases (see tests/test_oracle_*.py).
 */
#ifndef GDIST_ORACLE_H
#define GDIST_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Pose n float32 vertices: out[3i..3i+2] = ((R00 x + R01 y) + R02 z) + t0 ... */
void orc_pose_points(const float* v, int64_t n, const double pose[12], double* out);

/* Closest point on segment [a,b] to p; returns the distance, writes q. */
double orc_point_segment(const double p[3], const double a[3], const double b[3], double q[3]);

/* Closest point on closed triangle t (9 doubles) to p; returns distance. */
double orc_point_triangle(const double p[3], const double t[9], double q[3]);

/* Closest points of segments [p0,p1] and [q0,q1]; returns distance. */
double orc_segment_segment(const double p0[3], const double p1[3], const double q0[3],
                           const double q1[3], double cp[3], double cq[3]);

/* 1 if segment [p0,p1] crosses the plane of the non-degenerate triangle t at a
 * single point inside the closed triangle (x receives that point), else 0. */
int orc_segment_pierces(const double p0[3], const double p1[3], const double t[9], double x[3]);

/* Exact distance between closed triangles P and Q (9 doubles each).
 * cp / cq receive a closest point pair (may be NULL). */
double orc_tri_tri_min(const double P[9], const double Q[9], double cp[3], double cq[3]);

/* Largest distance between closed triangles P and Q (attained at vertices). */
double orc_tri_tri_max(const double P[9], const double Q[9], double cp[3], double cq[3]);

/* Box bounds (Sec. 4).  Boxes are {min x,y,z, max x,y,z}.  out[0] = conventional
 * lower bound of the min distance, out[1] = enhanced upper bound of the min
 * distance (literal 36 face-pair evaluation), out[2] = conventional upper bound
 * of the max distance (= conventional upper bound of the min distance),
 * out[3] = enhanced lower bound of the max distance (literal 36 face pairs). */
void orc_box_bounds(const double a[6], const double b[6], double out[4]);

/* Result of a mesh-pair query. */
typedef struct {
  double distance;     /* D_min or D_max                                         */
  int64_t tri_a;       /* canonical pair: lexicographically smallest (a,b) whose */
  int64_t tri_b;       /*   distance lies within tau of D                       */
  double point_a[3];   /* world-frame points on tri_a / tri_b for that pair     */
  double point_b[3];
  double pair_distance;/* distance of the canonical pair itself                 */
  int64_t n_ties;      /* number of pairs within tau of D                        */
  int64_t pairs_tested;/* triangle pairs evaluated                               */
} orc_result_t;

/* Brute force over all triangle pairs (mode 0 = min, 1 = max).  Splits A's
 * triangles over `threads` POSIX threads.  ties (may be NULL) receives up to
 * tie_cap (a,b) pairs of the tie set in lexicographic order.  Returns 0 on
 * success, nonzero on bad input. */
int orc_brute(const float* va, int64_t nva, const uint32_t* fa, int64_t nfa, const double pose_a[12],
              const float* vb, int64_t nvb, const uint32_t* fb, int64_t nfb, const double pose_b[12],
              int mode, double tau, int threads, orc_result_t* out, int64_t* ties, int64_t tie_cap);

/* Same contract, computed with the oracle's own median-split AABB tree and a
 * best-first search that prunes a node pair only when its conventional bound
 * is more than tau worse than the best value found (single-threaded). */
int orc_bvh(const float* va, int64_t nva, const uint32_t* fa, int64_t nfa, const double pose_a[12],
            const float* vb, int64_t nvb, const uint32_t* fb, int64_t nfb, const double pose_b[12],
            int mode, double tau, orc_result_t* out, int64_t* ties, int64_t tie_cap);

/* D_max by its plain definition restricted to vertices: max over vertex pairs. */
double orc_max_vertex_pairs(const float* va, int64_t nva, const double pose_a[12],
                            const float* vb, int64_t nvb, const double pose_b[12], int threads);

/* rowmax[i] = max over vertices b of B of |a_i - b| (posed), for every vertex a_i of A. */
void orc_vertex_row_max(const float* va, int64_t nva, const double pose_a[12],
                        const float* vb, int64_t nvb, const double pose_b[12], int threads, double* rowmax);

#ifdef __cplusplus
}
#endif
#endif
