/*
 * synth.c -- seeded synthetic point clouds (inputs only).
 *
 * This module generates input buffers and nothing else: it holds none of the
 * octree method's arithmetic.  Both the oracle and the GPU path consume the
 * buffers it writes.  Every value is a pure function of (seed, stream, index)
 * through the SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014),
 * so any slice of a cloud can be regenerated independently and in parallel.
 *
 * Record layout: float32 x, y, z; uint8 r, g, b, a (16 bytes), a = 255.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  float x, y, z;
  uint8_t r, g, b, a;
} spoint;

static const double PI = 3.14159265358979323846;

static uint64_t sm64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
/* 64 random bits for (seed, stream, index) */
static uint64_t rbits(uint64_t seed, uint64_t stream, uint64_t index) {
  return sm64(sm64(sm64(seed) ^ (stream * 0xD1B54A32D192ED03ull)) + index * 0x9E3779B97F4A7C15ull);
}
/* uniform in [0, 1) from the top 53 bits */
static double runif(uint64_t seed, uint64_t stream, uint64_t index) {
  return (double)(rbits(seed, stream, index) >> 11) * (1.0 / 9007199254740992.0);
}
static double rrange(uint64_t seed, uint64_t stream, uint64_t index, double lo, double hi) {
  return lo + (hi - lo) * runif(seed, stream, index);
}
/* standard normal by Box-Muller from two uniforms */
static double rnorm(uint64_t seed, uint64_t stream, uint64_t index) {
  double u1 = runif(seed, stream, 2 * index), u2 = runif(seed, stream, 2 * index + 1);
  return sqrt(-2.0 * log(1.0 - u1)) * cos(2.0 * PI * u2);
}
static uint8_t clamp8(double v) {
  if (v < 0.0) return 0;
  if (v > 255.0) return 255;
  return (uint8_t)v;
}
/* colour channel plus integer noise in -16..16 */
static uint8_t noisy(double base, uint64_t seed, uint64_t stream, uint64_t index) {
  int n = (int)(runif(seed, stream, index) * 33.0) - 16;
  return clamp8(floor(base + 0.5) + n);
}

/* streams */
enum { S_PARAM = 1, S_COMP, S_X, S_Y, S_Z, S_FACE, S_NOISE_R, S_NOISE_G, S_NOISE_B, S_PICK, S_GAUSS, S_U, S_V };

typedef struct {
  double amp, wavelength;
  double phi[4], psi[4];
} terrain_t;

static void terrain_init(terrain_t* t, uint64_t seed, uint64_t param_base, double amp, double wavelength) {
  t->amp = amp;
  t->wavelength = wavelength;
  for (int k = 0; k < 4; ++k) {
    t->phi[k] = rrange(seed, S_PARAM, param_base + 2 * k, 0.0, 2.0 * PI);
    t->psi[k] = rrange(seed, S_PARAM, param_base + 2 * k + 1, 0.0, 2.0 * PI);
  }
}
/* z = sum over 4 octaves of (A/2^k) sin(2 pi 2^k x / lambda + phi_k) cos(2 pi 2^k y / lambda + psi_k) */
static double terrain_z(const terrain_t* t, double x, double y) {
  double z = 0.0;
  for (int k = 0; k < 4; ++k) {
    double f = 2.0 * PI * (double)(1 << k) / t->wavelength;
    z += t->amp / (double)(1 << k) * sin(f * x + t->phi[k]) * cos(f * y + t->psi[k]);
  }
  return z;
}
/* height ramp (60,110,50) -> (150,120,80) -> (220,220,210) */
static void ramp(double tt, double c[3]) {
  static const double s0[3] = {60, 110, 50}, s1[3] = {150, 120, 80}, s2[3] = {220, 220, 210};
  if (tt < 0.0) tt = 0.0;
  if (tt > 1.0) tt = 1.0;
  for (int i = 0; i < 3; ++i)
    c[i] = tt < 0.5 ? s0[i] + (s1[i] - s0[i]) * (2.0 * tt) : s1[i] + (s2[i] - s1[i]) * (2.0 * tt - 1.0);
}

typedef struct {
  double cx, cy, w, d, h, z0;
  double col[3];
  double area_roof, area_wx, area_wy; /* roof, each wall along x, each wall along y */
} building_t;

typedef struct {
  double cx, cy, cz;
  double col[3];
} blob_t;

/* A tile: terrain + optional box buildings + optional Gaussian vegetation blobs. */
typedef struct {
  uint64_t seed;
  double ox, oy, side;
  double f_building, f_veg; /* fractions; terrain gets the rest */
  terrain_t ter;
  int nb;
  building_t* b;
  double* b_cum; /* cumulative building area */
  int nv;
  blob_t* v;
} tile_t;

static void tile_init(tile_t* t, uint64_t seed, double ox, double oy, double side, double amp, double wavelength,
                      double f_building, int nb, double f_veg, int nv) {
  memset(t, 0, sizeof(*t));
  t->seed = seed;
  t->ox = ox; t->oy = oy; t->side = side;
  t->f_building = nb > 0 ? f_building : 0.0;
  t->f_veg = nv > 0 ? f_veg : 0.0;
  terrain_init(&t->ter, seed, 0, amp, wavelength);
  t->nb = nb;
  if (nb > 0) {
    t->b = (building_t*)calloc((size_t)nb, sizeof(building_t));
    t->b_cum = (double*)calloc((size_t)nb, sizeof(double));
    double acc = 0.0;
    for (int j = 0; j < nb; ++j) {
      uint64_t pb = 1000 + 16ull * (uint64_t)j;
      building_t* B = &t->b[j];
      B->w = rrange(seed, S_PARAM, pb + 0, 10.0, 50.0);
      B->d = rrange(seed, S_PARAM, pb + 1, 10.0, 50.0);
      B->h = rrange(seed, S_PARAM, pb + 2, 5.0, 40.0);
      B->cx = rrange(seed, S_PARAM, pb + 3, 0.05 * side, 0.95 * side);
      B->cy = rrange(seed, S_PARAM, pb + 4, 0.05 * side, 0.95 * side);
      B->z0 = terrain_z(&t->ter, B->cx, B->cy);
      for (int c = 0; c < 3; ++c) B->col[c] = rrange(seed, S_PARAM, pb + 5 + (uint64_t)c, 80.0, 200.0);
      B->area_roof = B->w * B->d;
      B->area_wx = B->w * B->h;
      B->area_wy = B->d * B->h;
      acc += B->area_roof + 2.0 * B->area_wx + 2.0 * B->area_wy;
      t->b_cum[j] = acc;
    }
  }
  t->nv = nv;
  if (nv > 0) {
    t->v = (blob_t*)calloc((size_t)nv, sizeof(blob_t));
    for (int j = 0; j < nv; ++j) {
      uint64_t pb = 1000000 + 8ull * (uint64_t)j;
      blob_t* V = &t->v[j];
      V->cx = rrange(seed, S_PARAM, pb + 0, 0.0, side);
      V->cy = rrange(seed, S_PARAM, pb + 1, 0.0, side);
      V->cz = terrain_z(&t->ter, V->cx, V->cy) + rrange(seed, S_PARAM, pb + 2, 4.0, 12.0);
      V->col[0] = rrange(seed, S_PARAM, pb + 3, 40.0, 90.0);
      V->col[1] = rrange(seed, S_PARAM, pb + 4, 100.0, 160.0);
      V->col[2] = rrange(seed, S_PARAM, pb + 5, 30.0, 70.0);
    }
  }
}

static void tile_free(tile_t* t) {
  free(t->b); free(t->b_cum); free(t->v);
  memset(t, 0, sizeof(*t));
}

static void tile_point(const tile_t* t, uint64_t i, spoint* p) {
  const uint64_t s = t->seed;
  double u = runif(s, S_COMP, i);
  double x, y, z, col[3];
  if (u < t->f_building) {
    /* building: pick a building and a face proportionally to area */
    double a = runif(s, S_PICK, i) * t->b_cum[t->nb - 1];
    int lo = 0, hi = t->nb - 1;
    while (lo < hi) {
      int m = (lo + hi) / 2;
      if (t->b_cum[m] > a) hi = m; else lo = m + 1;
    }
    const building_t* B = &t->b[lo];
    double fa = runif(s, S_FACE, i) * (B->area_roof + 2.0 * B->area_wx + 2.0 * B->area_wy);
    double su = runif(s, S_U, i), sv = runif(s, S_V, i);
    double x0 = B->cx - 0.5 * B->w, y0 = B->cy - 0.5 * B->d;
    if (fa < B->area_roof) {
      x = x0 + su * B->w; y = y0 + sv * B->d; z = B->z0 + B->h;
    } else if ((fa -= B->area_roof) < 2.0 * B->area_wx) {
      x = x0 + su * B->w; y = fa < B->area_wx ? y0 : y0 + B->d; z = B->z0 + sv * B->h;
    } else {
      fa -= 2.0 * B->area_wx;
      y = y0 + su * B->d; x = fa < B->area_wy ? x0 : x0 + B->w; z = B->z0 + sv * B->h;
    }
    for (int c = 0; c < 3; ++c) col[c] = B->col[c];
  } else if (u < t->f_building + t->f_veg) {
    /* vegetation: isotropic Gaussian blob, sigma 2 m */
    int j = (int)(runif(s, S_PICK, i) * t->nv);
    if (j >= t->nv) j = t->nv - 1;
    const blob_t* V = &t->v[j];
    x = V->cx + 2.0 * rnorm(s, S_GAUSS, 3 * i);
    y = V->cy + 2.0 * rnorm(s, S_GAUSS, 3 * i + 1);
    z = V->cz + 2.0 * rnorm(s, S_GAUSS, 3 * i + 2);
    for (int c = 0; c < 3; ++c) col[c] = V->col[c];
  } else {
    /* terrain: uniform in the tile, height from the sine octaves, colour from height */
    x = runif(s, S_X, i) * t->side;
    y = runif(s, S_Y, i) * t->side;
    z = terrain_z(&t->ter, x, y);
    ramp((z + 1.875 * t->ter.amp) / (3.75 * t->ter.amp), col);
  }
  p->x = (float)(t->ox + x);
  p->y = (float)(t->oy + y);
  p->z = (float)z;
  p->r = noisy(col[0], s, S_NOISE_R, i);
  p->g = noisy(col[1], s, S_NOISE_G, i);
  p->b = noisy(col[2], s, S_NOISE_B, i);
  p->a = 255;
}

/* Generic tile; points [first, first+count) of the tile's sequence. */
int synth_tile(uint64_t seed, double ox, double oy, double side, double amp, double wavelength, double f_building,
               int n_buildings, double f_veg, int n_blobs, uint64_t first, uint64_t count, spoint* out) {
  tile_t t;
  tile_init(&t, seed, ox, oy, side, amp, wavelength, f_building, n_buildings, f_veg, n_blobs);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < (int64_t)count; ++k) tile_point(&t, first + (uint64_t)k, &out[k]);
  tile_free(&t);
  return 0;
}

/* ------------------------------------------------------- terrestrial scan */

typedef struct {
  int is_sphere;
  double c[3], r;        /* sphere */
  double n[3], u[3], v[3], w, h; /* rectangle: normal, in-plane axes, sides */
  double col[3];
  double area;
} prim_t;

int synth_scan(uint64_t seed, double box, int n_spheres, int n_planes, uint64_t first, uint64_t count, spoint* out) {
  int np = n_spheres + n_planes;
  prim_t* pr = (prim_t*)calloc((size_t)np, sizeof(prim_t));
  double* cum = (double*)calloc((size_t)np, sizeof(double));
  double acc = 0.0;
  for (int j = 0; j < np; ++j) {
    uint64_t pb = 5000 + 32ull * (uint64_t)j;
    prim_t* P = &pr[j];
    P->is_sphere = j < n_spheres;
    for (int a = 0; a < 3; ++a) P->c[a] = rrange(seed, S_PARAM, pb + (uint64_t)a, 0.1 * box, 0.9 * box);
    for (int a = 0; a < 3; ++a) P->col[a] = rrange(seed, S_PARAM, pb + 3 + (uint64_t)a, 40.0, 230.0);
    if (P->is_sphere) {
      P->r = rrange(seed, S_PARAM, pb + 6, 0.5, 8.0);
      P->area = 4.0 * PI * P->r * P->r;
    } else {
      /* random unit normal: normalised Gaussian vector */
      double g[3], len = 0.0;
      for (int a = 0; a < 3; ++a) { g[a] = rnorm(seed, S_PARAM, pb + 7 + (uint64_t)a); len += g[a] * g[a]; }
      len = sqrt(len);
      for (int a = 0; a < 3; ++a) P->n[a] = g[a] / len;
      /* in-plane axes: u = normalize(n x e), e the axis least aligned with n */
      double e[3] = {0, 0, 0};
      int m = fabs(P->n[0]) < fabs(P->n[1]) ? (fabs(P->n[0]) < fabs(P->n[2]) ? 0 : 2) : (fabs(P->n[1]) < fabs(P->n[2]) ? 1 : 2);
      e[m] = 1.0;
      double u[3] = {P->n[1] * e[2] - P->n[2] * e[1], P->n[2] * e[0] - P->n[0] * e[2], P->n[0] * e[1] - P->n[1] * e[0]};
      double lu = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
      for (int a = 0; a < 3; ++a) P->u[a] = u[a] / lu;
      P->v[0] = P->n[1] * P->u[2] - P->n[2] * P->u[1];
      P->v[1] = P->n[2] * P->u[0] - P->n[0] * P->u[2];
      P->v[2] = P->n[0] * P->u[1] - P->n[1] * P->u[0];
      P->w = rrange(seed, S_PARAM, pb + 10, 5.0, 40.0);
      P->h = rrange(seed, S_PARAM, pb + 11, 5.0, 40.0);
      P->area = P->w * P->h;
    }
    acc += P->area;
    cum[j] = acc;
  }
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < (int64_t)count; ++k) {
    uint64_t i = first + (uint64_t)k;
    double a = runif(seed, S_PICK, i) * acc;
    int lo = 0, hi = np - 1;
    while (lo < hi) {
      int m = (lo + hi) / 2;
      if (cum[m] > a) hi = m; else lo = m + 1;
    }
    const prim_t* P = &pr[lo];
    double pos[3], nrm[3];
    double noise = 0.001 * rnorm(seed, S_GAUSS, i);
    if (P->is_sphere) {
      /* uniform on the sphere: z uniform in [-1,1], angle uniform */
      double zz = 2.0 * runif(seed, S_U, i) - 1.0, ph = 2.0 * PI * runif(seed, S_V, i);
      double rr = sqrt(1.0 - zz * zz);
      nrm[0] = rr * cos(ph); nrm[1] = rr * sin(ph); nrm[2] = zz;
      for (int q = 0; q < 3; ++q) pos[q] = P->c[q] + P->r * nrm[q];
    } else {
      double su = (runif(seed, S_U, i) - 0.5) * P->w, sv = (runif(seed, S_V, i) - 0.5) * P->h;
      for (int q = 0; q < 3; ++q) { pos[q] = P->c[q] + su * P->u[q] + sv * P->v[q]; nrm[q] = P->n[q]; }
    }
    for (int q = 0; q < 3; ++q) {
      double c = pos[q] + noise * nrm[q];
      if (c < 0.0) c = 0.0;
      if (c > box) c = box;
      pos[q] = c;
    }
    spoint* p = &out[k];
    p->x = (float)pos[0]; p->y = (float)pos[1]; p->z = (float)pos[2];
    p->r = noisy(P->col[0], seed, S_NOISE_R, i);
    p->g = noisy(P->col[1], seed, S_NOISE_G, i);
    p->b = noisy(P->col[2], seed, S_NOISE_B, i);
    p->a = 255;
  }
  free(pr); free(cum);
  return 0;
}

/* uniforms / normals for host-side planning (chunk sizes, arrivals) */
void synth_uniform(uint64_t seed, uint64_t stream, uint64_t first, uint64_t count, double* out) {
  for (uint64_t k = 0; k < count; ++k) out[k] = runif(seed, stream, first + k);
}
void synth_normal(uint64_t seed, uint64_t stream, uint64_t first, uint64_t count, double* out) {
  for (uint64_t k = 0; k < count; ++k) out[k] = rnorm(seed, stream, first + k);
}
