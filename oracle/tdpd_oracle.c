/*
 * tdpd_oracle.c -- CPU oracle for one time step of transport dissipative
 * particle dynamics (tDPD) with red-blood-cell (RBC) membranes, after
 * Blumers et al., "GPU-accelerated red blood cells simulations with transport
 * dissipative particle dynamics" (arXiv:1611.06163).
 *
 * TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark are the only callers; the product library
 * never links, loads or calls this code and shares nothing with it.
 *
 * It is plain and slow on purpose.  Arithmetic is FP64 on the FP32 state
 * handed in, sums are the sums the paper writes:
 *   - force on particle i: Eq. (2), sum over j of Eqs. (3)-(5) with the
 *     fluctuation-dissipation pairing of Eq. (6);
 *   - concentration rate: Eq. (7) with the Fickian and random fluxes of
 *     Eqs. (8)-(9), the pairing of Eq. (10) and the source term Q^S (read as
 *     a zero-order source less a first-order decay per species and type);
 *   - membrane: WLC and POW bond potentials, Eqs. (13)-(14), bond viscosity
 *     and its random partner, Eqs. (15)-(16), area and volume constraints,
 *     Eqs. (17)-(18), bending, Eq. (19);
 *   - time integration: velocity Verlet (the paper gives only the ODEs,
 *     Eqs. (1)-(2)).
 * Readings of points the paper leaves open are stated with the code that
 * takes them.
 *
 * The only FP32 arithmetic is the pair predicate (which particles are within
 * a cutoff), evaluated exactly as specified so that pair sets can be compared
 * bit for bit:  per axis d = fl(x_j - x_i), except across the periodic
 * boundary (|x_j - x_i| > L/2), where the coordinate nearer 0 is lifted by L
 * first: d = fl(fl(x_j + L) - x_i) or fl(x_j - fl(x_i + L)); d2 =
 * fmaf(dz,dz,fmaf(dy,dy,dx*dx)), pair iff 0 < d2 < fl(rcut*rcut).  The rule
 * is symmetric: d_ji = -d_ij bit for bit.  Build with -ffp-contract=off.
 *
 * Random numbers: Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
 * implemented here from its published definition.  Counter (k, min gid,
 * max gid, box_id<<8 | stream), key (seed_lo, seed_hi); uniforms
 * u = (2*(bits>>9)+1) * 2^-24; normals by Box-Muller, sqrt(-2 ln u0)
 * cos(2 pi u1) from a pair of words (and sqrt(-2 ln u0) sin(2 pi u1) where two
 * normals per pair are drawn).  Stream 0 gives the pair force noise xi (cos
 * of words 0,1) and the species-0 flux noise (cos of words 2,3); stream m>=1
 * gives species 2m-1 and 2m the same way; streams 64, 65, 66 give twelve
 * normals (cos, sin of words 0,1, then cos, sin of words 2,3, per stream),
 * the first nine of which are the membrane bond's Wiener matrix, row major.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXT 4
#define ORC_MAXS 16
#define ORC_MAXMESH 16

/* terms bitmask */
#define T_CONS   1
#define T_DISS   2
#define T_RAND   4
#define T_FICK   8
#define T_FRAND  16
#define T_BOND   32
#define T_BVISC  64
#define T_BRAND  128
#define T_AREA   256
#define T_VOL    512
#define T_BEND   1024
#define T_BODY   2048

/* error bits */
#define E_OVEREXT 1
#define E_NONFINITE 2

#define FROZEN_BIT (1u << 8)

typedef struct {
  float box[3];
  float rc, rcc;
  double dt, kT, rho, m_s, s_exp, sc_exp;
  int32_t n_types, n_species;
  double alpha[ORC_MAXT * ORC_MAXT];
  double gamma[ORC_MAXT * ORC_MAXT];
  double sigma[ORC_MAXT * ORC_MAXT];
  double kappa[ORC_MAXS * ORC_MAXT * ORC_MAXT];
  double body_force[3];
  int32_t wall_axis;
  double wall_w;
  uint32_t seed_lo, seed_hi, box_id;
  int32_t terms;
  float shear_rate; /* Lees-Edwards shear rate (0: plain periodic box) */
  /* source term of Eq. (7): Q^S_i = source[s*T + t_i] - decay[s*T + t_i] C_i */
  double source[ORC_MAXS * ORC_MAXT];
  double decay[ORC_MAXS * ORC_MAXT];
  double wall_radius; /* wall_axis 3: cylinder about the x-parallel axis */
} orc_params;

typedef struct {
  double p, x0, m_pow, kb, theta0, kg, kl, kv, gamma_t, gamma_c;
} orc_mesh_params;

typedef struct {
  int nv, ntri, nedge, ndih;
  int32_t *tri;   /* [ntri][3] */
  int32_t *edge;  /* [nedge][2], a < b */
  int32_t *dih;   /* [ndih][4] = a, b, c, d ; triangles (a,b,c) and (d,c,b) */
  int32_t *bfs;   /* [nv][2] = vertex, parent (parent -1 for the root) */
  double *l0, *lm, *kp, *A0t;
  double A0, V0, theta0;
  orc_mesh_params mp;
} orc_mesh;

typedef struct {
  orc_params p;
  int nmesh;
  orc_mesh mesh[ORC_MAXMESH];
  int nrbc, caprbc;
  int32_t *rbc_mesh;
  int64_t *rbc_first;
} orc_sys;

/* ------------------------------------------------------------------ RNG */

static void philox_round(uint32_t c[4], uint32_t k0, uint32_t k1) {
  /* one Philox-4x32 round: two 32x32->64 products, their high halves xored
     with the other two counter words and the key, low halves passed on */
  const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
  const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  const uint32_t n0 = hi1 ^ c[1] ^ k0;
  const uint32_t n2 = hi0 ^ c[3] ^ k1;
  c[0] = n0;
  c[1] = lo1;
  c[2] = n2;
  c[3] = lo0;
}

void orc_philox4x32(const uint32_t ctr[4], const uint32_t key[2], int rounds,
                    uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < rounds; ++r) {
    if (r > 0) { /* key schedule: Weyl sequence */
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    philox_round(c, k0, k1);
  }
  memcpy(out, c, sizeof(c));
}

double orc_u01(uint32_t bits) {
  return ((double)(bits >> 9) * 2.0 + 1.0) * (1.0 / 16777216.0);
}

static double box_muller(uint32_t a, uint32_t b) {
  return sqrt(-2.0 * log(orc_u01(a))) * cos(2.0 * M_PI * orc_u01(b));
}

/* two standard normals for the unordered pair {gi, gj} at step k */
void orc_pair_normals(const orc_params *p, uint32_t k, uint32_t gi, uint32_t gj,
                      uint32_t stream, double out[2]) {
  const uint32_t lo = gi < gj ? gi : gj, hi = gi < gj ? gj : gi;
  const uint32_t ctr[4] = {k, lo, hi, (p->box_id << 8) | stream};
  const uint32_t key[2] = {p->seed_lo, p->seed_hi};
  uint32_t w[4];
  orc_philox4x32(ctr, key, 10, w);
  out[0] = box_muller(w[0], w[1]);
  out[1] = box_muller(w[2], w[3]);
}

/* four standard normals for the unordered pair: Box-Muller cos and sin of
   words (0,1), then of words (2,3) */
void orc_pair_normals4(const orc_params *p, uint32_t k, uint32_t gi, uint32_t gj,
                       uint32_t stream, double out[4]) {
  const uint32_t lo = gi < gj ? gi : gj, hi = gi < gj ? gj : gi;
  const uint32_t ctr[4] = {k, lo, hi, (p->box_id << 8) | stream};
  const uint32_t key[2] = {p->seed_lo, p->seed_hi};
  uint32_t w[4];
  orc_philox4x32(ctr, key, 10, w);
  for (int h = 0; h < 2; ++h) {
    const double r = sqrt(-2.0 * log(orc_u01(w[2 * h])));
    const double a = 2.0 * M_PI * orc_u01(w[2 * h + 1]);
    out[2 * h] = r * cos(a);
    out[2 * h + 1] = r * sin(a);
  }
}

/* ------------------------------------------------------------ predicate */

/* Box geometry at step counter k.  With a shear rate (reading C21, Lees-
   Edwards boundaries) the periodic image of the box above (y + L_y) is
   displaced by delta_k in x and moves with +u = shear L_y in x:
     u = fl32(shear * L_y), delta_k = fl32(fmod(shear L_y * (k dt), L_x))
   with the products taken in FP64 from the FP32 parameters (the library
   uses the same sequence). */
typedef struct {
  float L[3];
  float delta, u;
  int le;
} geom_t;

static geom_t geom_at(const orc_params *p, uint32_t k) {
  geom_t g;
  for (int a = 0; a < 3; ++a) g.L[a] = p->box[a];
  g.le = p->shear_rate != 0.0f;
  g.delta = 0.0f;
  g.u = 0.0f;
  if (g.le) {
    const double a = (double)p->shear_rate * (double)p->box[1];
    const double b = (double)k * (double)(float)p->dt;
    g.u = (float)a;
    g.delta = (float)fmod(a * b, (double)p->box[0]);
    if (g.delta >= p->box[0]) g.delta = 0.0f;
  }
  return g;
}

/* FP32 displacement d = x_j - x_i at the nearest image (reading C4) and its
   squared length.  For a pair across the periodic boundary of an axis the
   coordinate nearer 0 is lifted by +L (one rounding, the same from both
   sides), so d_ji = -d_ij exactly.  In a sheared box a pair across the y
   boundary lifts the particle with the smaller y into the image above: y by
   +L_y and x by delta + m L_x, where X1 = fl(x + delta) and m in {-2,..,1}
   brings X1 nearest the other particle's x (decided from dx1 = fl(x_o - X1)
   in FP32, again the same from both sides); x and z of such a pair use the
   lifted coordinates, z the plain rule.  s (may be NULL) gets the shift of
   x_j's image relative to x_i's image (the exact-arithmetic displacement is
   x_j + s - x_i) and *sv (may be NULL) the x-velocity offset of x_j's image
   relative to x_i's (v_ij = v_i - v_j - sv). */
static float disp_geo(const float *xi, const float *xj, const geom_t *g, float d[3], double s[3],
                      double *sv) {
  int lift = 0; /* 1: x_i lifted into the image above, 2: x_j lifted */
  if (g->le) {
    const float ry = xj[1] - xi[1];
    if (ry > 0.5f * g->L[1]) lift = 1;
    else if (ry < -0.5f * g->L[1]) lift = 2;
  }
  if (sv) *sv = 0.0;
  for (int a = 0; a < 3; ++a) {
    const float L = g->L[a];
    double sh = 0.0;
    if (lift && a < 2) {
      const float *xl = lift == 1 ? xi : xj, *xo = lift == 1 ? xj : xi;
      float X;
      double shl; /* lifted coordinate and its exact shift */
      if (a == 1) {
        X = xl[1] + L;
        shl = L;
      } else {
        const float X1 = xl[0] + g->delta;
        const float dx1 = xo[0] - X1;
        int m = 0;
        if (dx1 > 0.5f * L) m = 1;
        else if (dx1 < -0.5f * L) m = (dx1 + L < -0.5f * L) ? -2 : -1;
        X = X1 + (float)m * L;
        shl = (double)g->delta + (double)m * (double)L;
      }
      if (lift == 1) {
        d[a] = xo[a] - X;
        sh = -shl;
      } else {
        d[a] = X - xo[a];
        sh = shl;
      }
      if (s) s[a] = sh;
      continue;
    }
    const float raw = xj[a] - xi[a];
    const float half = 0.5f * L;
    if (raw > half) {          /* x_i near 0: lift x_i */
      sh = -L;
      const float xl = xi[a] + L;
      d[a] = xj[a] - xl;
    } else if (raw < -half) {  /* x_j near 0: lift x_j */
      sh = L;
      const float xl = xj[a] + L;
      d[a] = xl - xi[a];
    } else {
      d[a] = raw;
    }
    if (s) s[a] = sh;
  }
  if (sv && lift) *sv = lift == 2 ? (double)g->u : -(double)g->u;
  return fmaf(d[2], d[2], fmaf(d[1], d[1], d[0] * d[0]));
}

/* ------------------------------------------------------------ cell list */

typedef struct {
  int n[3];
  int *head, *next;
  int brute;
} cells_t;

static void cells_build(cells_t *c, const orc_params *p, int n, const float *xf) {
  const double rmax = p->rc > p->rcc ? p->rc : p->rcc;
  c->brute = 0;
  for (int a = 0; a < 3; ++a) {
    c->n[a] = (int)floor((double)p->box[a] / (rmax * 1.01));
    if (c->n[a] < 3) c->brute = 1;
  }
  c->head = NULL;
  c->next = NULL;
  if (c->brute) return;
  const long nc = (long)c->n[0] * c->n[1] * c->n[2];
  c->head = (int *)malloc(sizeof(int) * nc);
  c->next = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
  for (long q = 0; q < nc; ++q) c->head[q] = -1;
  /* insert in descending index order so each bucket lists ascending indices */
  for (int i = n - 1; i >= 0; --i) {
    int ci[3];
    for (int a = 0; a < 3; ++a) {
      int v = (int)floor((double)xf[3 * i + a] * c->n[a] / (double)p->box[a]);
      if (v < 0) v = 0;
      if (v >= c->n[a]) v = c->n[a] - 1;
      ci[a] = v;
    }
    const long q = ((long)ci[2] * c->n[1] + ci[1]) * c->n[0] + ci[0];
    c->next[i] = c->head[q];
    c->head[q] = i;
  }
}

static void cells_free(cells_t *c) {
  free(c->head);
  free(c->next);
}

static void cell_of(const cells_t *c, const float *box, const float *x, int ci[3]) {
  for (int a = 0; a < 3; ++a) {
    int v = (int)floor((double)x[a] * c->n[a] / (double)box[a]);
    if (v < 0) v = 0;
    if (v >= c->n[a]) v = c->n[a] - 1;
    ci[a] = v;
  }
}

/* Collect all j != i with 0 < d2 < rcut2 into list (indices), returns count.
   list must hold n entries.  In a sheared box a neighbour row across the y
   boundary is searched over its whole x extent (its cells are displaced by
   delta in x). */
static int neighbours(const cells_t *c, const geom_t *g, int n, const float *xf,
                      int i, float rcut2, int *list, int *nzero) {
  int m = 0;
  float d[3];
  if (c->brute) {
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      const float d2 = disp_geo(xf + 3 * i, xf + 3 * j, g, d, NULL, NULL);
      if (d2 == 0.0f) { if (nzero) ++*nzero; continue; }
      if (d2 < rcut2) list[m++] = j;
    }
    return m;
  }
  int ci[3];
  cell_of(c, g->L, xf + 3 * i, ci);
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy) {
      const int cyr = ci[1] + dy;
      const int across = g->le && (cyr < 0 || cyr >= c->n[1]);
      const int x0 = across ? 0 : -1, x1 = across ? c->n[0] - 1 : 1;
      for (int dx = x0; dx <= x1; ++dx) {
        const int cx = across ? dx : (ci[0] + dx + c->n[0]) % c->n[0];
        const int cy = (cyr + c->n[1]) % c->n[1];
        const int cz = (ci[2] + dz + c->n[2]) % c->n[2];
        const long q = ((long)cz * c->n[1] + cy) * c->n[0] + cx;
        for (int j = c->head[q]; j >= 0; j = c->next[j]) {
          if (j == i) continue;
          const float d2 = disp_geo(xf + 3 * i, xf + 3 * j, g, d, NULL, NULL);
          if (d2 == 0.0f) { if (nzero) ++*nzero; continue; }
          if (d2 < rcut2) list[m++] = j;
        }
      }
    }
  return m;
}

/* ------------------------------------------------------------- system */

orc_sys *orc_create(const orc_params *p) {
  orc_sys *s = (orc_sys *)calloc(1, sizeof(orc_sys));
  s->p = *p;
  return s;
}

void orc_set_params(orc_sys *s, const orc_params *p) { s->p = *p; }

void orc_destroy(orc_sys *s) {
  if (!s) return;
  for (int m = 0; m < s->nmesh; ++m) {
    orc_mesh *M = &s->mesh[m];
    free(M->tri); free(M->edge); free(M->dih); free(M->bfs);
    free(M->l0); free(M->lm); free(M->kp); free(M->A0t);
  }
  free(s->rbc_mesh);
  free(s->rbc_first);
  free(s);
}

static void sub3(const double *a, const double *b, double *o) {
  o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2];
}
static void cross3(const double *a, const double *b, double *o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double *a, const double *b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static double norm3(const double *a) { return sqrt(dot3(a, a)); }

/* signed angle between the outward normals of triangles (a,b,c) and (d,c,b);
   positive where the surface is convex (bends away from its outward side) */
static double dihedral_theta(const double *a, const double *b, const double *c,
                             const double *d) {
  double ba[3], ca[3], cd[3], bd[3], n1[3], n2[3], e[3], x[3];
  sub3(b, a, ba); sub3(c, a, ca); cross3(ba, ca, n1);
  sub3(c, d, cd); sub3(b, d, bd); cross3(cd, bd, n2);
  sub3(c, b, e);
  cross3(n1, n2, x);
  return atan2(dot3(x, e) / norm3(e), dot3(n1, n2));
}

/* gradient of dihedral_theta with respect to a, b, c, d */
static void dihedral_grad(const double *a, const double *b, const double *c,
                          const double *d, double g[4][3]) {
  double ba[3], ca[3], cd[3], bd[3], n1[3], n2[3], e[3], ab[3], db[3];
  sub3(b, a, ba); sub3(c, a, ca); cross3(ba, ca, n1);
  sub3(c, d, cd); sub3(b, d, bd); cross3(cd, bd, n2);
  sub3(c, b, e);
  const double le2 = dot3(e, e), le = sqrt(le2);
  const double f1 = -le / dot3(n1, n1), f2 = -le / dot3(n2, n2);
  sub3(a, b, ab); sub3(d, b, db);
  const double ta = dot3(ab, e) / le2, td = dot3(db, e) / le2;
  for (int q = 0; q < 3; ++q) {
    const double ga = f1 * n1[q], gd = f2 * n2[q];
    g[0][q] = ga;
    g[3][q] = gd;
    g[1][q] = (ta - 1.0) * ga + (td - 1.0) * gd;
    g[2][q] = -ta * ga - td * gd;
  }
}

/* Register a membrane mesh: triangles (outward counter-clockwise) and its
   reference (rest) shape.  Rest quantities, the readings of Section 2.2:
   per-bond rest length l0 from the reference shape, maximum extension
   l_m = l0/x0, POW coefficient k_p per bond chosen so that the WLC and POW
   forces cancel at l0 (stress-free bonds); A_{0,j} the reference triangle
   areas, A_0 their sum, V_0 the reference volume; theta0 the given value or,
   if NaN, the mean reference dihedral angle.  Returns the mesh id or < 0. */
int orc_add_mesh(orc_sys *s, int nv, int ntri, const int32_t *tri, const double *ref,
                 const orc_mesh_params *mp) {
  if (s->nmesh >= ORC_MAXMESH || nv < 4 || ntri < 4) return -1;
  orc_mesh *M = &s->mesh[s->nmesh];
  memset(M, 0, sizeof(*M));
  M->nv = nv;
  M->ntri = ntri;
  M->mp = *mp;
  M->tri = (int32_t *)malloc(sizeof(int32_t) * 3 * ntri);
  memcpy(M->tri, tri, sizeof(int32_t) * 3 * ntri);
  /* directed-edge table: owner[a*nv+b] = triangle holding edge a->b */
  int *owner = (int *)malloc(sizeof(int) * (size_t)nv * nv);
  for (long q = 0; q < (long)nv * nv; ++q) owner[q] = -1;
  for (int t = 0; t < ntri; ++t)
    for (int e = 0; e < 3; ++e) {
      const int a = tri[3 * t + e], b = tri[3 * t + (e + 1) % 3];
      if (a < 0 || a >= nv || b < 0 || b >= nv || owner[(long)a * nv + b] >= 0) {
        free(owner);
        return -2; /* not a consistently oriented manifold */
      }
      owner[(long)a * nv + b] = t;
    }
  M->edge = (int32_t *)malloc(sizeof(int32_t) * 3 * ntri);
  M->dih = (int32_t *)malloc(sizeof(int32_t) * 6 * ntri);
  for (int a = 0; a < nv; ++a)
    for (int b = a + 1; b < nv; ++b) {
      const int t1 = owner[(long)a * nv + b], t2 = owner[(long)b * nv + a];
      if (t1 < 0 && t2 < 0) continue;
      if (t1 < 0 || t2 < 0) { free(owner); return -3; } /* open edge */
      M->edge[2 * M->nedge] = a;
      M->edge[2 * M->nedge + 1] = b;
      M->nedge++;
      /* dihedral over edge b0->c0 of t1 = (a0, b0, c0) and t2 = (d0, c0, b0) */
      int a0 = -1, d0 = -1;
      for (int e = 0; e < 3; ++e) {
        if (tri[3 * t1 + e] != a && tri[3 * t1 + e] != b) a0 = tri[3 * t1 + e];
        if (tri[3 * t2 + e] != a && tri[3 * t2 + e] != b) d0 = tri[3 * t2 + e];
      }
      int32_t *D = M->dih + 4 * M->ndih;
      D[0] = a0; D[1] = a; D[2] = b; D[3] = d0; /* t1 holds a->b */
      M->ndih++;
    }
  free(owner);
  /* breadth-first order over the edge graph, used to unwrap periodic images */
  M->bfs = (int32_t *)malloc(sizeof(int32_t) * 2 * nv);
  {
    int *seen = (int *)calloc(nv, sizeof(int));
    int qh = 0, qt = 0;
    M->bfs[0] = 0; M->bfs[1] = -1; seen[0] = 1; qt = 1;
    while (qh < qt) {
      const int v = M->bfs[2 * qh];
      ++qh;
      for (int e = 0; e < M->nedge; ++e) {
        int w = -1;
        if (M->edge[2 * e] == v) w = M->edge[2 * e + 1];
        else if (M->edge[2 * e + 1] == v) w = M->edge[2 * e];
        if (w >= 0 && !seen[w]) {
          seen[w] = 1;
          M->bfs[2 * qt] = w;
          M->bfs[2 * qt + 1] = v;
          ++qt;
        }
      }
    }
    free(seen);
    if (qt != nv) return -4; /* not connected */
  }
  M->l0 = (double *)malloc(sizeof(double) * M->nedge);
  M->lm = (double *)malloc(sizeof(double) * M->nedge);
  M->kp = (double *)malloc(sizeof(double) * M->nedge);
  M->A0t = (double *)malloc(sizeof(double) * ntri);
  const double kT = s->p.kT;
  for (int e = 0; e < M->nedge; ++e) {
    double d[3];
    sub3(ref + 3 * M->edge[2 * e + 1], ref + 3 * M->edge[2 * e], d);
    const double l0 = norm3(d), x0 = mp->x0;
    M->l0[e] = l0;
    M->lm[e] = l0 / x0;
    const double fw = kT / mp->p * (0.25 / ((1 - x0) * (1 - x0)) - 0.25 + x0);
    M->kp[e] = fw * pow(l0, mp->m_pow);
  }
  M->A0 = 0;
  M->V0 = 0;
  for (int t = 0; t < ntri; ++t) {
    const double *a = ref + 3 * tri[3 * t], *b = ref + 3 * tri[3 * t + 1],
                 *c = ref + 3 * tri[3 * t + 2];
    double ba[3], ca[3], n[3], bc[3];
    sub3(b, a, ba); sub3(c, a, ca); cross3(ba, ca, n);
    M->A0t[t] = 0.5 * norm3(n);
    M->A0 += M->A0t[t];
    cross3(b, c, bc);
    M->V0 += dot3(a, bc) / 6.0;
  }
  if (isnan(mp->theta0)) {
    double sum = 0;
    for (int q = 0; q < M->ndih; ++q) {
      const int32_t *D = M->dih + 4 * q;
      sum += dihedral_theta(ref + 3 * D[0], ref + 3 * D[1], ref + 3 * D[2], ref + 3 * D[3]);
    }
    M->theta0 = sum / M->ndih;
  } else {
    M->theta0 = mp->theta0;
  }
  return s->nmesh++;
}

/* out: A0, V0, theta0, nedge, ndih, ntri */
void orc_mesh_info(const orc_sys *s, int mesh, double *out) {
  const orc_mesh *M = &s->mesh[mesh];
  out[0] = M->A0; out[1] = M->V0; out[2] = M->theta0;
  out[3] = M->nedge; out[4] = M->ndih; out[5] = M->ntri;
}

void orc_mesh_topology(const orc_sys *s, int mesh, int32_t *edge, int32_t *dih) {
  const orc_mesh *M = &s->mesh[mesh];
  if (edge) memcpy(edge, M->edge, sizeof(int32_t) * 2 * M->nedge);
  if (dih) memcpy(dih, M->dih, sizeof(int32_t) * 4 * M->ndih);
}

int orc_add_rbc(orc_sys *s, int mesh, int64_t first_gid) {
  if (mesh < 0 || mesh >= s->nmesh) return -1;
  if (s->nrbc == s->caprbc) {
    s->caprbc = s->caprbc ? 2 * s->caprbc : 16;
    s->rbc_mesh = (int32_t *)realloc(s->rbc_mesh, sizeof(int32_t) * s->caprbc);
    s->rbc_first = (int64_t *)realloc(s->rbc_first, sizeof(int64_t) * s->caprbc);
  }
  s->rbc_mesh[s->nrbc] = mesh;
  s->rbc_first[s->nrbc] = first_gid;
  return s->nrbc++;
}

/* body id of every particle: the RBC it belongs to, -1 otherwise */
static int32_t *make_body(const orc_sys *s, int n) {
  int32_t *body = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
  for (int i = 0; i < n; ++i) body[i] = -1;
  for (int r = 0; r < s->nrbc; ++r) {
    const int nv = s->mesh[s->rbc_mesh[r]].nv;
    for (int v = 0; v < nv; ++v) {
      const int64_t g = s->rbc_first[r] + v;
      if (g >= 0 && g < n) body[g] = r;
    }
  }
  return body;
}

/* ------------------------------------------------------- pair enumeration */

/* All unordered pairs (i < j) with 0 < d2 < fl(rcut^2) under the FP32 rule.
   which = 0: rcut = rc, 1: rcut = rcc.  brute = 1 forces the O(N^2) scan.
   Writes up to cap pairs, returns the total count through *count and the
   number of coincident (d2 == 0) ordered pairs through *nzero. */
void orc_pairs(const orc_sys *s, int64_t n, const float *xf, int which, int brute, uint32_t k,
               int64_t cap, int32_t *out, int64_t *count, int64_t *nzero) {
  const orc_params *p = &s->p;
  const geom_t g = geom_at(p, k);
  const float rcut = which ? p->rcc : p->rc;
  const float rcut2 = rcut * rcut;
  cells_t c;
  cells_build(&c, p, (int)n, xf);
  if (brute) c.brute = 1;
  int *list = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
  int64_t m = 0;
  int nz = 0;
  for (int i = 0; i < n; ++i) {
    const int cnt = neighbours(&c, &g, (int)n, xf, i, rcut2, list, &nz);
    for (int q = 0; q < cnt; ++q) {
      const int j = list[q];
      if (j <= i) continue;
      if (m < cap) {
        out[2 * m] = i;
        out[2 * m + 1] = j;
      }
      ++m;
    }
  }
  free(list);
  cells_free(&c);
  *count = m;
  *nzero = nz;
}

/* ------------------------------------------------------------- membrane */

static double wrap_delta(double d, double L) { return d - L * nearbyint(d / L); }

/* Unwrapped coordinates of RBC r's vertices: breadth-first along bonds, each
   bond taken at its nearest periodic image (in a sheared box a bond across
   the y boundary takes the sheared image: x shifted by delta, and the
   vertex's x velocity by u, which uvx [nv] accumulates). */
static void unwrap_rbc(const orc_sys *s, const geom_t *g, int r, const double *pos, double *u,
                       double *uvx) {
  const orc_mesh *M = &s->mesh[s->rbc_mesh[r]];
  const int64_t g0 = s->rbc_first[r];
  for (int q = 0; q < M->nv; ++q) {
    const int v = M->bfs[2 * q], par = M->bfs[2 * q + 1];
    const double *xv = pos + 3 * (g0 + v);
    if (par < 0) {
      for (int a = 0; a < 3; ++a) u[3 * v + a] = xv[a];
      uvx[v] = 0.0;
      continue;
    }
    const double *xp = pos + 3 * (g0 + par);
    int ny = 0; /* +1: v is taken in the image above its parent, -1: below */
    if (g->le) {
      const double dy = xv[1] - xp[1];
      if (dy > 0.5 * g->L[1]) ny = -1;
      else if (dy < -0.5 * g->L[1]) ny = 1;
    }
    const double shx = ny * (double)g->delta;
    u[3 * v] = u[3 * par] + wrap_delta(xv[0] + shx - xp[0], (double)g->L[0]);
    u[3 * v + 1] = u[3 * par + 1] + (xv[1] + ny * (double)g->L[1] - xp[1]);
    if (!g->le) u[3 * v + 1] = u[3 * par + 1] + wrap_delta(xv[1] - xp[1], (double)g->L[1]);
    u[3 * v + 2] = u[3 * par + 2] + wrap_delta(xv[2] - xp[2], (double)g->L[2]);
    uvx[v] = uvx[par] + ny * (double)g->u;
  }
}

/* Membrane forces (added into F, indexed by gid), energies (bond, area,
   volume, bending) and per-RBC total area and volume. */
static double vnorm(const double *v) { return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

static int membrane(const orc_sys *s, int64_t n, const double *pos, const double *vel,
                    uint32_t k, double *F, double *energy, double *av, double *Fabs) {
  const orc_params *p = &s->p;
  const int terms = p->terms;
  const geom_t g = geom_at(p, k);
  int err = 0;
  for (int r = 0; r < s->nrbc; ++r) {
    const orc_mesh *M = &s->mesh[s->rbc_mesh[r]];
    const orc_mesh_params *mp = &M->mp;
    const int64_t g0 = s->rbc_first[r];
    if (g0 < 0 || g0 + M->nv > n) return -1;
    double *u = (double *)malloc(sizeof(double) * 3 * M->nv);
    double *uvx = (double *)malloc(sizeof(double) * M->nv);
    double *f = (double *)calloc(3 * M->nv, sizeof(double));
    double *fab = (double *)calloc(M->nv, sizeof(double));
    unwrap_rbc(s, &g, r, pos, u, uvx);
    const double *vv = vel + 3 * g0;
    /* bonds, Eqs. (13)-(16) */
    for (int e = 0; e < M->nedge; ++e) {
      const int a = M->edge[2 * e], b = M->edge[2 * e + 1];
      double d[3];
      sub3(u + 3 * b, u + 3 * a, d); /* a -> b */
      const double l = norm3(d);
      double fa[3] = {0, 0, 0};
      double fmag = 0; /* sum of the magnitudes of the parts added below */
      if (terms & T_BOND) {
        const double x = l / M->lm[e];
        if (x >= 1.0) {
          err |= E_OVEREXT;
        } else {
          /* dU/dl of WLC and POW; positive pulls a toward b */
          const double dwlc = p->kT / mp->p * (0.25 / ((1 - x) * (1 - x)) - 0.25 + x);
          const double dpow = -M->kp[e] / pow(l, mp->m_pow);
          for (int q = 0; q < 3; ++q) fa[q] += (dwlc + dpow) * d[q] / l;
          fmag += fabs(dwlc) + fabs(dpow);
          if (energy) {
            energy[0] += p->kT * M->lm[e] / (4 * mp->p) * x * x * (3 - 2 * x) / (1 - x);
            if (mp->m_pow != 1.0)
              energy[0] += M->kp[e] / ((mp->m_pow - 1) * pow(l, mp->m_pow - 1));
            else
              energy[0] += -M->kp[e] * log(l);
          }
        }
      }
      /* e_ab points from b to a (the paper's e_ij = r_ij / |r_ij|) */
      const double eab[3] = {-d[0] / l, -d[1] / l, -d[2] / l};
      if (terms & T_BVISC) {
        double vab[3];
        sub3(vv + 3 * a, vv + 3 * b, vab);
        vab[0] += uvx[a] - uvx[b];
        const double ve = dot3(vab, eab);
        for (int q = 0; q < 3; ++q) fa[q] += -mp->gamma_t * vab[q] - mp->gamma_c * ve * eab[q];
        fmag += mp->gamma_t * vnorm(vab) + mp->gamma_c * fabs(ve);
      }
      if (terms & T_BRAND) {
        double W[12];
        for (int t = 0; t < 3; ++t)
          orc_pair_normals4(p, k, (uint32_t)(g0 + a), (uint32_t)(g0 + b), 64 + t, W + 4 * t);
        double WS[9];
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) WS[3 * i + j] = 0.5 * (W[3 * i + j] + W[3 * j + i]);
        const double trS = WS[0] + WS[4] + WS[8];
        const double trW = W[0] + W[4] + W[8];
        const double ct = sqrt(2 * mp->gamma_t);
        const double cc = sqrt(fmax(3 * mp->gamma_c - mp->gamma_t, 0.0)) / 3.0;
        const double amp = sqrt(2 * p->kT / p->dt);
        for (int i = 0; i < 3; ++i) {
          double acc = 0;
          for (int j = 0; j < 3; ++j) {
            double Mij = ct * (WS[3 * i + j] - (i == j ? trS / 3.0 : 0.0));
            if (i == j) Mij += cc * trW;
            acc += Mij * eab[j];
          }
          fa[i] += amp * acc;
          fmag += fabs(amp * acc);
        }
      }
      for (int q = 0; q < 3; ++q) {
        f[3 * a + q] += fa[q];
        f[3 * b + q] -= fa[q];
      }
      fab[a] += fmag;
      fab[b] += fmag;
    }
    /* area and volume, Eqs. (17)-(18) */
    double At = 0, Vt = 0;
    for (int t = 0; t < M->ntri; ++t) {
      const double *a = u + 3 * M->tri[3 * t], *b = u + 3 * M->tri[3 * t + 1],
                   *c = u + 3 * M->tri[3 * t + 2];
      double ba[3], ca[3], nn[3], bc[3];
      sub3(b, a, ba); sub3(c, a, ca); cross3(ba, ca, nn);
      At += 0.5 * norm3(nn);
      cross3(b, c, bc);
      Vt += dot3(a, bc) / 6.0;
    }
    if (av) {
      av[2 * r] = At;
      av[2 * r + 1] = Vt;
    }
    const double cg = mp->kg * (At - M->A0) / M->A0;
    const double cv = mp->kv * (Vt - M->V0) / M->V0;
    if (energy) {
      if (terms & T_AREA) energy[1] += mp->kg * (At - M->A0) * (At - M->A0) / (2 * M->A0);
      if (terms & T_VOL) energy[2] += mp->kv * (Vt - M->V0) * (Vt - M->V0) / (2 * M->V0);
    }
    for (int t = 0; t < M->ntri; ++t) {
      const int ia = M->tri[3 * t], ib = M->tri[3 * t + 1], ic = M->tri[3 * t + 2];
      const double *a = u + 3 * ia, *b = u + 3 * ib, *c = u + 3 * ic;
      double ba[3], ca[3], nn[3];
      sub3(b, a, ba); sub3(c, a, ca); cross3(ba, ca, nn);
      const double nl = norm3(nn), At_ = 0.5 * nl;
      const double nh[3] = {nn[0] / nl, nn[1] / nl, nn[2] / nl};
      if (terms & T_AREA) {
        const double cl = mp->kl * (At_ - M->A0t[t]) / M->A0t[t];
        if (energy) energy[1] += mp->kl * (At_ - M->A0t[t]) * (At_ - M->A0t[t]) / (2 * M->A0t[t]);
        /* dA/da = 1/2 n x (c - b), cyclic */
        const double *P[3] = {a, b, c};
        const int I[3] = {ia, ib, ic};
        for (int v = 0; v < 3; ++v) {
          double opp[3], g[3];
          sub3(P[(v + 2) % 3], P[(v + 1) % 3], opp);
          cross3(nh, opp, g);
          for (int q = 0; q < 3; ++q) f[3 * I[v] + q] -= (cg + cl) * 0.5 * g[q];
          /* Error scale of this term: the global coefficient itself (A^t is
             a sum of exact triangle areas, so c_g carries only its own
             rounding), the local triangle area A_j and its rest value A_0j
             (separately rounded), times the gradient's size 1/2 |c - b|,
             which does not depend on where the cell sits. */
          fab[I[v]] += (fabs(cg) + mp->kl * (At_ + M->A0t[t]) / M->A0t[t]) * 0.5 * vnorm(g);
        }
      }
      if (terms & T_VOL) {
        /* dV_t/da = 1/6 b x c, cyclic (the same vector for every origin:
           1/6 (b - a) x (c - a) at a); error scale |c_v| |dV_t/da| */
        double g[3];
        cross3(b, c, g);
        for (int q = 0; q < 3; ++q) f[3 * ia + q] -= cv * g[q] / 6.0;
        cross3(c, a, g);
        for (int q = 0; q < 3; ++q) f[3 * ib + q] -= cv * g[q] / 6.0;
        cross3(a, b, g);
        for (int q = 0; q < 3; ++q) f[3 * ic + q] -= cv * g[q] / 6.0;
        for (int v = 0; v < 3; ++v) fab[M->tri[3 * t + v]] += fabs(cv) * nl / 6.0;
      }
    }
    /* bending, Eq. (19) */
    if (terms & T_BEND) {
      for (int q = 0; q < M->ndih; ++q) {
        const int32_t *D = M->dih + 4 * q;
        const double *P[4] = {u + 3 * D[0], u + 3 * D[1], u + 3 * D[2], u + 3 * D[3]};
        const double th = dihedral_theta(P[0], P[1], P[2], P[3]);
        double g[4][3];
        dihedral_grad(P[0], P[1], P[2], P[3], g);
        const double coef = -mp->kb * sin(th - M->theta0);
        if (energy) energy[3] += mp->kb * (1 - cos(th - M->theta0));
        for (int v = 0; v < 4; ++v) {
          for (int a = 0; a < 3; ++a) f[3 * D[v] + a] += coef * g[v][a];
          /* sin(theta - theta0) = sin cos0 - cos sin0, two rounded terms */
          fab[D[v]] += mp->kb * (fabs(sin(th) * cos(M->theta0)) + fabs(cos(th) * sin(M->theta0))) *
                       vnorm(g[v]);
        }
      }
    }
    for (int v = 0; v < M->nv; ++v) {
      for (int a = 0; a < 3; ++a) F[3 * (g0 + v) + a] += f[3 * v + a];
      if (Fabs) Fabs[g0 + v] += fab[v];
    }
    free(u);
    free(uvx);
    free(f);
    free(fab);
  }
  return err;
}

/* ------------------------------------------------------------------ forces */

static double powp(double w, double e) { return w > 0 ? pow(w, e) : 0.0; }

/* Force F_i (Eq. 2) and concentration rate Q_i (Eq. 7) of every particle
   selected by `which` (NULL = all), at step counter k.  Frozen particles get
   F = Q = 0.  Pair forces are skipped between vertices of the same RBC (the
   bonded terms act there); fluxes act between every pair.  Membrane forces
   and the body force are added for every particle.  av (may be NULL) gets
   per-RBC (A, V).  Returns error bits (or < 0). */
int orc_forces(const orc_sys *s, int64_t n64, const double *pos, const double *vel,
               const double *conc, const uint32_t *flags, uint32_t k,
               const uint8_t *which, double *F, double *Q, double *av,
               double *energy, int64_t *nzero_out, double *Fabs, double *Qabs,
               double *Fmabs) {
  const orc_params *p = &s->p;
  const int n = (int)n64, S = p->n_species, T = p->n_types;
  const int terms = p->terms;
  float *xf = (float *)malloc(sizeof(float) * 3 * (n > 0 ? n : 1));
  for (int i = 0; i < 3 * n; ++i) xf[i] = (float)pos[i];
  int32_t *body = make_body(s, n);
  cells_t c;
  cells_build(&c, p, n, xf);
  const float rc2 = p->rc * p->rc, rcc2 = p->rcc * p->rcc;
  const float rmax2 = rc2 > rcc2 ? rc2 : rcc2;
  const double isdt = 1.0 / sqrt(p->dt);
  const geom_t g = geom_at(p, k);
  int64_t nzero = 0;
#pragma omp parallel reduction(+ : nzero)
  {
    int *list = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
#pragma omp for schedule(dynamic, 64)
    for (int i = 0; i < n; ++i) {
      double *Fi = F + 3 * i, *Qi = Q + (size_t)S * i;
      Fi[0] = Fi[1] = Fi[2] = 0;
      for (int sp = 0; sp < S; ++sp) Qi[sp] = 0;
      if (Fabs) Fabs[i] = 0;
      if (Qabs)
        for (int sp = 0; sp < S; ++sp) Qabs[(size_t)S * i + sp] = 0;
      if (which && !which[i]) continue;
      if (flags[i] & FROZEN_BIT) continue;
      int nz = 0;
      const int m = neighbours(&c, &g, n, xf, i, rmax2, list, &nz);
      nzero += nz;
      const int ti = (int)(flags[i] & 0xffu);
      for (int q = 0; q < m; ++q) {
        const int j = list[q];
        const int tj = (int)(flags[j] & 0xffu);
        float df[3];
        double sh[3], sv;
        const float d2 = disp_geo(xf + 3 * i, xf + 3 * j, &g, df, sh, &sv);
        /* FP64 displacement x_j - x_i at the same periodic image */
        double d[3];
        for (int a = 0; a < 3; ++a) d[a] = (pos[3 * j + a] + sh[a]) - pos[3 * i + a];
        const double r = norm3(d);
        const double e[3] = {-d[0] / r, -d[1] / r, -d[2] / r}; /* e_ij, j -> i */
        if (d2 < rc2 && !(body[i] >= 0 && body[i] == body[j])) {
          const double w = 1.0 - r / p->rc;
          double fs = 0;
          if (terms & T_CONS) fs += p->alpha[ti * T + tj] * w;
          if (terms & T_DISS) {
            double vij[3];
            sub3(vel + 3 * i, vel + 3 * j, vij);
            vij[0] -= sv; /* velocity of x_j's sheared image */
            fs += -p->gamma[ti * T + tj] * powp(w, p->s_exp) * dot3(e, vij);
          }
          if (terms & T_RAND) {
            double z[2];
            orc_pair_normals(p, k, (uint32_t)i, (uint32_t)j, 0, z);
            fs += p->sigma[ti * T + tj] * powp(w, 0.5 * p->s_exp) * z[0] * isdt;
          }
          for (int a = 0; a < 3; ++a) Fi[a] += fs * e[a];
          if (Fabs) Fabs[i] += fabs(fs);
        }
        if (d2 < rcc2) {
          const double wc = 1.0 - r / p->rcc;
          for (int sp = 0; sp < S; ++sp) {
            const double kap = p->kappa[(sp * T + ti) * T + tj];
            const double ci = conc[(size_t)S * i + sp], cj = conc[(size_t)S * j + sp];
            if (terms & T_FICK) {
              const double qd = -kap * powp(wc, p->sc_exp) * (ci - cj);
              Qi[sp] += qd;
              if (Qabs) Qabs[(size_t)S * i + sp] += fabs(qd);
            }
            if ((terms & T_FRAND) && p->m_s > 0) {
              const double eps = p->m_s * sqrt(kap * p->rho * fmax(ci + cj, 0.0));
              double z[2];
              const int stream = (sp + 1) / 2, word = (sp + 1) % 2;
              orc_pair_normals(p, k, (uint32_t)i, (uint32_t)j, (uint32_t)stream, z);
              /* zeta_ij = -zeta_ji: the draw belongs to the lower gid */
              const double zeta = (i < j) ? z[word] : -z[word];
              const double qr = eps * powp(wc, 0.5 * p->sc_exp) * isdt * zeta;
              Qi[sp] += qr;
              if (Qabs) Qabs[(size_t)S * i + sp] += fabs(qr);
            }
          }
        }
      }
      /* Q^S of Eq. (7), the external contribution the paper leaves open
         (reading: a zero-order source and a first-order decay of the
         particle's own concentration, per species and particle type) */
      for (int sp = 0; sp < S; ++sp) {
        const double a = p->source[sp * T + ti], kd = p->decay[sp * T + ti];
        if (a == 0 && kd == 0) continue;
        const double ci = conc[(size_t)S * i + sp];
        Qi[sp] += a - kd * ci;
        if (Qabs) Qabs[(size_t)S * i + sp] += fabs(a) + fabs(kd * ci);
      }
      if (terms & T_BODY) {
        for (int a = 0; a < 3; ++a) Fi[a] += p->body_force[a];
        if (Fabs) Fabs[i] += sqrt(p->body_force[0] * p->body_force[0] +
                                  p->body_force[1] * p->body_force[1] +
                                  p->body_force[2] * p->body_force[2]);
      }
    }
    free(list);
  }
  cells_free(&c);
  int err = 0;
  if (s->nrbc > 0) {
    double *Fm = (double *)calloc(3 * (size_t)(n > 0 ? n : 1), sizeof(double));
    double *Fma = (Fabs || Fmabs) ? (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double))
                                  : NULL;
    err = membrane(s, n, pos, vel, k, Fm, energy, av, Fma);
    if (err >= 0)
      for (int i = 0; i < n; ++i) {
        if ((which && !which[i]) || (flags[i] & FROZEN_BIT)) continue;
        for (int a = 0; a < 3; ++a) F[3 * i + a] += Fm[3 * i + a];
        if (Fabs) Fabs[i] += Fma[i];
        if (Fmabs) Fmabs[i] = Fma[i];
      }
    free(Fm);
    free(Fma);
  }
  for (int i = 0; i < 3 * n && err >= 0; ++i)
    if (!isfinite(F[i])) err |= E_NONFINITE;
  free(xf);
  free(body);
  if (nzero_out) *nzero_out = nzero;
  return err;
}

/* membrane-only energies (bond, area, volume, bending) and forces */
int orc_membrane(const orc_sys *s, int64_t n, const double *pos, const double *vel,
                 uint32_t k, double *F, double *energy, double *av) {
  for (int64_t i = 0; i < 3 * n; ++i) F[i] = 0;
  if (energy) energy[0] = energy[1] = energy[2] = energy[3] = 0;
  return membrane(s, n, pos, vel, k, F, energy, av, NULL);
}

/* ------------------------------------------------------------- integrator */

static double wrap_pos(double x, double L) {
  if (x < 0) x += L;
  if (x >= L) x -= L;
  if (x >= L || x < 0) x = 0; /* only reachable by rounding */
  return x;
}

/* One velocity-Verlet step (reading of Eqs. 1-2 and 7): half kick of v and C
   with the stored F and Q, drift, wall reflection, periodic wrap, new F and
   Q at step counter k (the dissipative force sees the half-step velocity),
   second half kick.  Frozen particles neither move nor change C.  In place. */
int orc_step(const orc_sys *s, int64_t n64, double *pos, double *vel, double *conc,
             double *F, double *Q, const uint32_t *flags, uint32_t k, double *av) {
  const orc_params *p = &s->p;
  const int n = (int)n64, S = p->n_species;
  const double h = 0.5 * p->dt;
  const geom_t g = geom_at(p, k); /* positions after the drift are at step k */
  for (int i = 0; i < n; ++i) {
    if (flags[i] & FROZEN_BIT) continue;
    for (int a = 0; a < 3; ++a) vel[3 * i + a] += h * F[3 * i + a];
    for (int sp = 0; sp < S; ++sp) conc[(size_t)S * i + sp] += h * Q[(size_t)S * i + sp];
    for (int a = 0; a < 3; ++a) pos[3 * i + a] += p->dt * vel[3 * i + a];
    if (p->wall_axis == 3) {
      /* cylindrical wall (reading of the tube of the paper's transport
         validation): a mobile particle that ends the drift farther than R
         from the axis (y, z) = (L_y/2, L_z/2) is mirrored through the
         cylinder along its radius, r -> 2R - r, and its velocity reversed */
      const double cy = 0.5 * p->box[1], cz = 0.5 * p->box[2], R = p->wall_radius;
      double *x = pos + 3 * i;
      const double dy = x[1] - cy, dz = x[2] - cz, r = sqrt(dy * dy + dz * dz);
      if (r > R) {
        const double f = (2 * R - r) / r;
        x[1] = cy + dy * f;
        x[2] = cz + dz * f;
        for (int q = 0; q < 3; ++q) vel[3 * i + q] = -vel[3 * i + q];
      }
    } else if (p->wall_axis >= 0) {
      const int a = p->wall_axis;
      const double L = p->box[a], w = p->wall_w;
      double *x = pos + 3 * i + a;
      int hit = 0;
      if (*x < w) { *x = 2 * w - *x; hit = 1; }
      else if (*x > L - w) { *x = 2 * (L - w) - *x; hit = 1; }
      if (hit)
        for (int q = 0; q < 3; ++q) vel[3 * i + q] = -vel[3 * i + q];
    }
    if (g.le) {
      /* crossing the y boundary of a sheared box: into the image below or
         above, x by -/+ delta and the x velocity by -/+ u */
      double *x = pos + 3 * i;
      if (x[1] >= p->box[1]) {
        x[1] -= p->box[1];
        x[0] -= (double)g.delta;
        vel[3 * i] -= (double)g.u;
      } else if (x[1] < 0) {
        x[1] += p->box[1];
        x[0] += (double)g.delta;
        vel[3 * i] += (double)g.u;
      }
    }
    for (int a = 0; a < 3; ++a) pos[3 * i + a] = wrap_pos(pos[3 * i + a], p->box[a]);
  }
  const int err =
      orc_forces(s, n, pos, vel, conc, flags, k, NULL, F, Q, av, NULL, NULL, NULL, NULL, NULL);
  for (int i = 0; i < n; ++i) {
    if (flags[i] & FROZEN_BIT) continue;
    for (int a = 0; a < 3; ++a) vel[3 * i + a] += h * F[3 * i + a];
    for (int sp = 0; sp < S; ++sp) conc[(size_t)S * i + sp] += h * Q[(size_t)S * i + sp];
  }
  return err;
}

/* Diagnostics: out[0..2] total momentum of mobile particles (m = 1),
   out[3] kT = sum |v - vbar|^2 / (3 (N_mobile - 1)), out[4..4+S) total
   concentration per species. */
void orc_diag(const orc_sys *s, int64_t n, const double *vel, const double *conc,
              const uint32_t *flags, double *out) {
  const int S = s->p.n_species;
  double P[3] = {0, 0, 0}, v2 = 0;
  int64_t nm = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (flags[i] & FROZEN_BIT) continue;
    ++nm;
    for (int a = 0; a < 3; ++a) {
      P[a] += vel[3 * i + a];
      v2 += vel[3 * i + a] * vel[3 * i + a];
    }
  }
  out[0] = P[0]; out[1] = P[1]; out[2] = P[2];
  out[3] = nm > 1 ? (v2 - dot3(P, P) / (double)nm) / (3.0 * (nm - 1)) : 0.0;
  for (int sp = 0; sp < S; ++sp) {
    double c = 0;
    for (int64_t i = 0; i < n; ++i) c += conc[(size_t)S * i + sp];
    out[4 + sp] = c;
  }
}

/* normals for a batch of pairs (RNG statistics tests) */
void orc_pair_normals_batch(const orc_params *p, uint32_t k, int64_t n, const uint32_t *gi,
                            const uint32_t *gj, uint32_t stream, double *out) {
  for (int64_t q = 0; q < n; ++q) orc_pair_normals(p, k, gi[q], gj[q], stream, out + 2 * q);
}

/* FP32 displacement of x_j seen from x_i (tests of the predicate rule) */
float orc_disp(const orc_sys *s, const float *xi, const float *xj, uint32_t k, float *d) {
  const geom_t g = geom_at(&s->p, k);
  return disp_geo(xi, xj, &g, d, NULL, NULL);
}
