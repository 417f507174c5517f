/* C ABI of the FP64 CPU oracle of the bound-driven caustic estimator.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously correct CPU
 * definition the GPU library is checked against.  Only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark may load it; the product
 * path never does.  It shares no code, header or constant with the HIP
 * library (the two meet only through seeded inputs).
 *
 * Conventions: every array is FP64, structure-of-arrays, owned by the caller.
 * Functions return 0 (or a count >= 0) on success and a negative value on bad
 * arguments.  Tuples are numbered emitter * n_tri + triangle; for two
 * reflections (emitter * n_tri + t1) * n_tri2 + t2.
 */
#ifndef CAUSTIC_ORACLE_H
#define CAUSTIC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t chain;     /* 0 = one reflection (R), 1 = one refraction (T), 2 = two reflections (RR) */
  int64_t n_tri;     /* specular triangles of the first surface */
  const double* pos; /* [9][n_tri]: p0.xyz, p1.xyz, p2.xyz */
  const double* nrm; /* [9][n_tri]: n0.xyz, n1.xyz, n2.xyz (vertex normals) */
  int64_t n_tri2;    /* RR: second surface */
  const double* pos2;
  const double* nrm2;
  double eta;        /* T: ratio of indices of refraction, incident over transmitted */
  double q0[3], f1[3], f2[3]; /* receiver x = q0 + u f1 + v f2, (u,v) in [0,1]^2 */
  int64_t n_emit;
  const double* epos; /* [3][n_emit] */
  const double* eI;   /* [n_emit] intensities */
  /* area lights (one reflection only): NULL for point lights, else [6][n_emit]
   * edges a, b of parallelogram emitters x0 = epos + z1 a + z2 b, (z1, z2) in
   * [0,1]^2, every point of which emits with intensity eI; the irradiance is
   * the mean over (z1, z2) */
  const double* eedge;
} orc_scene;

typedef struct {
  int32_t max_depth;   /* subdivision depth cap, counted from the initialised root box */
  double sigma;        /* stop when the clipped position-bound area is below sigma */
  double alpha;        /* stop when E_hi / E_lo < alpha (E_lo > 0) */
  int32_t grid_res;    /* G: receiver grid is G x G cells over [0,1]^2 */
  int32_t init_pieces; /* domain initialisation keeps at most this many boxes */
  int32_t init_levels; /* and descends at most this many levels */
  int32_t flags;       /* bit 0: fixed depth (only the depth cap stops);
                          bit 1: no remainder variable (ablation, T only);
                          bit 2: refraction irradiance bound by implicit
                          differentiation (T only) */
  double cover_frac;   /* a tuple whose leaves' cell rectangles add up to at
                          least cover_frac * G^2 cells is stored once, in the
                          cover-all list, with the largest E_hi of its leaves,
                          instead of in the cells; 0 disables the list */
} orc_params;

/* Path evaluation at barycentric (u, v) of a tuple.  out[0..9] =
 * u_k, v_k, t, E_k, detJ, admissible (0/1), beta (T), x1.x, x1.y, x1.z */
int orc_eval_path(const orc_scene* s, int64_t tuple, double u, double v, double* out);
/* The same from the point (z1, z2) of an area emitter. */
int orc_eval_path_at(const orc_scene* s, int64_t tuple, double u, double v, double z1, double z2, double* out);

/* Bound of one box [u0,u1]x[v0,v1] of a tuple's barycentric domain.
 * out[0] = 1 if the box is live, 0 if it is culled;
 * out[1..4] = u_lo, u_hi, v_lo, v_hi of the position bound clipped to [0,1]^2;
 * out[5..6] = E_lo, E_hi (E_hi may be +inf); out[7] = 1 if the position bound
 * was universal.  want_irr = 0 skips the irradiance bound (E = [0, inf)). */
int orc_box_bound(const orc_scene* s, int64_t tuple, const double* box, int want_irr, double* out);
/* The same with build flags (4: the refraction irradiance bound by implicit
 * differentiation). */
int orc_box_bound_flags(const orc_scene* s, int64_t tuple, const double* box, int want_irr, int flags,
                        double* out);

/* Full precomputation: tuples, domain initialisation, adaptive subdivision,
 * leaves and the receiver grid. */
void* orc_build(const orc_scene* s, const orc_params* p, int n_threads);
void orc_free(void* h);
int64_t orc_n_leaves(const void* h);
/* leaves: tuple[n], code[n][3] = depth, iu, iv (box index at that depth inside
 * the tuple's root box), box[n][4] = u0,u1,v0,v1, ukbox[n][4] = u_lo,u_hi,v_lo,v_hi,
 * E[n][2] = E_lo, E_hi */
int orc_get_leaves(const void* h, int64_t* tuple, int32_t* code, double* box, double* ukbox, double* E);
int64_t orc_n_roots(const void* h);
/* root boxes after domain initialisation: tuple[n], box[n][4] */
int orc_get_roots(const void* h, int64_t* tuple, double* box);
/* stats[0..8] = tuples, live tuples, boxes bounded, leaves, grid entries
 * (the cells' entries plus the cover-all list), infinite-bound leaves,
 * universal-position leaves, max leaves of one tuple, cover-all tuples */
int orc_build_stats(const void* h, double* stats);
/* The list stored in grid cell (cu, cv): tuples ascending with their
 * per-tuple bound E~.  Returns the list length (writes at most cap entries). */
int64_t orc_cell_list(const void* h, int32_t cu, int32_t cv, int64_t* tuples, double* Et, int64_t cap);
/* The cover-all list: tuples ascending with the largest E_hi of their leaves.
 * A shading point's candidate list U is its cell's list followed by this one. */
int64_t orc_cover_list(const void* h, int64_t* tuples, double* Et, int64_t cap);

/* Estimator of Alg. 1 at each shading point (points [3][n]).
 * mode 0: sample with the bound-optimal probabilities, roots by Newton from the
 *         covering leaves;  mode 1: exhaustive (every tuple of U with P = 1),
 *         same roots;  mode 2/3: as 0/1 with brute-force roots.
 * mode | 4:  uniform P = W'/|U| instead of the bound-optimal P;
 * mode | 8:  one-sample estimator with P1 = E~ / sum E~, W draws;
 * mode | 12: bound-optimal P, one sample per next-fit bin of total P <= 1
 *         (these three exclude mode 1; -1 for that combination).
 * stats (nullable) [n][4] = |U|, |S|, roots found, sum over U of E~^2 / P. */
int orc_query(const void* h, const double* pts, int64_t n, double W, uint64_t seed, int mode,
              double* E_out, double* stats, int n_threads);

/* Reference irradiance: brute-force roots of every admissible tuple, ignoring
 * all bounds (multi-start Newton from a barycentric lattice of resolution
 * `lattice`). */
int orc_true_irradiance(const orc_scene* s, const double* pts, int64_t n, int lattice, double* E_out,
                        int n_threads);
/* Brute-force roots of one tuple at one shading point: roots[k][4] = u, v, E_k, residual. */
int64_t orc_tuple_roots(const orc_scene* s, int64_t tuple, const double* x, int lattice, double* roots,
                        int64_t cap);
/* Tuple construction of two reflections (Sec. 6.1): the second-surface
 * triangles t2 that form a candidate pair with first triangle t1 under
 * emitter e (light in front of t1, and the interval test of the pair), in
 * ascending order.  Returns the count (writes at most cap). */
int64_t orc_pair_list(const orc_scene* s, int64_t emitter, int64_t t1, int64_t* t2_out, int64_t cap);
/* Roots of one tuple found from the covering leaves of a build. */
int64_t orc_tuple_roots_leaves(const void* h, int64_t tuple, const double* x, double* roots, int64_t cap);

/* The candidates one shading point selects from a list U[n] with bounds Et[n]
 * (sampler 0 Alg. 1 with the bound-optimal P, 1 uniform, 2 one-sample, 3 bins;
 * as orc_query modes 0, 4, 8, 12): indices into the list and the weight P of
 * each (contribution E(T) / P).  Returns the count (writes at most cap). */
int64_t orc_sample(const double* Et, const int64_t* U, int64_t n, double W, uint64_t seed, uint64_t point,
                   int sampler, int64_t* k_out, double* P_out, int64_t cap);

/* Smallest distance between a decision quantity of that selection and its
 * threshold (|r - P|; |r S - C_k| / S for the one-sample running sums; |fill +
 * P - 1| and the interval ends for the bins).  Negative on bad arguments. */
double orc_sample_margin(const double* Et, const int64_t* U, int64_t n, double W, uint64_t seed, uint64_t point,
                         int sampler);

/* Bound-optimal selection probabilities for a candidate list with bounds Et[n]
 * and expected sample count W (Sec. 5.4 with the water-filling solve of gamma). */
int orc_probabilities(const double* Et, int64_t n, double W, double* P);
/* Counter-based generator Philox4x32-10 (Salmon et al., SC 2011). */
void orc_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out);
/* The uniform in [0,1) drawn for (seed, point index, tuple). */
double orc_uniform(uint64_t seed, uint64_t point, uint32_t tuple);

/* Bernstein primitives exposed for unit tests; deg arrays have 4 entries. */
int orc_bern_mul(const int32_t* da, const double* a, const int32_t* db, const double* b, double* out);
int orc_bern_elevate(const int32_t* da, const double* a, const int32_t* dto, double* out);
int orc_bern_deriv(const int32_t* da, const double* a, int axis, double* out);
int orc_bern_split(const int32_t* da, const double* a, int axis, double t, double* left, double* right);
double orc_bern_eval(const int32_t* da, const double* a, const double* x);
/* Degree reduction (Sec. 6.1): least-squares approximant of degree dto <= da
   (SVD of the elevation matrix per reduced axis) and in *rem the largest
   residual coefficient at degree da.  Returns -1 when dto exceeds da. */
int orc_bern_reduce(const int32_t* da, const double* a, const int32_t* dto, double* out, double* rem);
/* out[0] = kind (0 direct [lo,hi], 1 split (-inf,lo]U[hi,inf), 2 unbounded), out[1] = lo, out[2] = hi */
int orc_ratio_bound(const int32_t* dp, const double* p, const int32_t* dq, const double* q, double* out);
/* Secant approximation of sqrt on [blo, bhi] (0 < blo <= bhi):
 * out = a, b, delta_lo, delta_hi with sqrt(x) - (a x + b) in [delta_lo, delta_hi]. */
int orc_sqrt_secant(double blo, double bhi, double* out);

#ifdef __cplusplus
}
#endif
#endif
