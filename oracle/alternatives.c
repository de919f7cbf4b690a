/* Valid results of the descent (and of uniform stepping) under near-ties
 * (test infrastructure).
 *
 * The descent takes discrete decisions: which texels the ray crosses, which of
 * them has the smallest lower bound, where the half-texel samples sit, which
 * sample has the smallest clearance.  When a decision's FP64 margin is below
 * what single precision can resolve, either outcome is a correct evaluation of
 * the method.  This file walks every such branch and returns the set of
 * angular clearances the method can yield for one ray.  With all tolerances at
 * zero it walks exactly the one path of oracle.c (the pins check this).
 *
 * It never reads anything produced by the GPU path.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle_internal.h"

#define ALT_MAXVALS 256
#define ALT_MAXPIECES 24
#define ALT_MAXVARIANTS 64

typedef struct {
  const ray_t* r;
  double eh_abs, eh_rel;  /* height tolerance: eh_abs + eh_rel * t (metres) */
  double et_abs, et_rel;  /* position tolerance: et_abs + et_rel * t/delta (texels) */
  long budget;
  int overflow;
} alt_t;

static double eps_h(const alt_t* A, double t) { return A->eh_abs + A->eh_rel * fabs(t); }
static double eps_t(const alt_t* A, double t) {
  return A->et_abs + A->et_rel * fabs(t) / A->r->s->delta;
}

typedef struct {
  double v[ALT_MAXVALS];
  int n;
} valset;

static void vs_add(alt_t* A, valset* s, double v) {
  for (int k = 0; k < s->n; ++k)
    if (s->v[k] == v) return;
  if (s->n >= ALT_MAXVALS) {
    A->overflow = 1;
    return;
  }
  s->v[s->n++] = v;
}

typedef struct {
  int cx, cy;
  double t0, t1;
  int kind;          /* 0 fixed, 1 optional (near an end), 2 corner */
  int acx, acy;      /* corner: the other cell the ray may clip first */
} piece_t;

/* Nominal pieces of the ray between lo and hi at level m, with the corner
 * ambiguity of near-simultaneous x/y crossings flagged. */
static int build_pieces(const ray_t* r, int m, double ta, double tb, double w, piece_t* pc) {
  double S = ldexp(1.0, m);
  double lo = ta - w, hi = tb + w;
  double qa[2], qb[2], Hd;
  or_ray_point(r, lo, &qa[0], &qa[1], &Hd);
  or_ray_point(r, hi, &qb[0], &qb[1], &Hd);
  double et[2 * OR_MAXCAND + 2];
  int ea[2 * OR_MAXCAND + 2];
  int ne = 0;
  for (int a = 0; a < 2; ++a) {
    double l = qa[a] < qb[a] ? qa[a] : qb[a];
    double h = qa[a] < qb[a] ? qb[a] : qa[a];
    for (double k = floor(l / S) + 1.0; k * S < h; k += 1.0) {
      double t = or_t_on_line(r, a, k * S);
      if (t < lo) t = lo;
      if (t > hi) t = hi;
      if (ne < 2 * OR_MAXCAND) {
        et[ne] = t;
        ea[ne] = a;
        ne++;
      }
    }
  }
  /* insertion sort by time */
  for (int k = 1; k < ne; ++k) {
    double t = et[k];
    int a = ea[k], q = k - 1;
    while (q >= 0 && et[q] > t) {
      et[q + 1] = et[q];
      ea[q + 1] = ea[q];
      q--;
    }
    et[q + 1] = t;
    ea[q + 1] = a;
  }
  double bt[2 * OR_MAXCAND + 4];
  int ba[2 * OR_MAXCAND + 4];
  int nb = 0;
  bt[nb] = lo;
  ba[nb++] = -1;
  for (int k = 0; k < ne; ++k) {
    bt[nb] = et[k];
    ba[nb++] = ea[k];
  }
  bt[nb] = hi;
  ba[nb++] = -1;
  int np = 0;
  int sgn[2] = {or_motion_sign(r, 0), or_motion_sign(r, 1)};
  for (int k = 0; k + 1 < nb; ++k) {
    double u = bt[k], v = bt[k + 1];
    int closepair = w > 0.0 && ba[k] >= 0 && ba[k + 1] >= 0 && ba[k] != ba[k + 1] && (v - u) < w;
    if (!(v > u) && !closepair) continue;
    double qx, qy;
    or_ray_point(r, 0.5 * (u + v), &qx, &qy, &Hd);
    int cx = (int)floor(qx / S), cy = (int)floor(qy / S);
    if (closepair) {
      /* the cell before crossing ba[k]: step back across it */
      int px = cx, py = cy;
      if (!(v > u)) {
        /* zero-length corner: the midpoint lies on both lines; recover the
         * cell before both crossings from the previous piece */
        if (np > 0) {
          px = pc[np - 1].cx;
          py = pc[np - 1].cy;
        }
      } else {
        if (ba[k] == 0) px -= sgn[0];
        else py -= sgn[1];
      }
      /* nominal: cross ba[k] first; other: cross ba[k+1] first */
      int nx = px, ny = py, ox = px, oy = py;
      if (ba[k] == 0) nx += sgn[0];
      else ny += sgn[1];
      if (ba[k + 1] == 0) ox += sgn[0];
      else oy += sgn[1];
      if (np < ALT_MAXPIECES) {
        pc[np].cx = nx;
        pc[np].cy = ny;
        pc[np].t0 = u;
        pc[np].t1 = v;
        pc[np].kind = (v > u) ? 2 : 3; /* 3: corner absent nominally */
        pc[np].acx = ox;
        pc[np].acy = oy;
        np++;
      }
      continue;
    }
    if (np > 0 && pc[np - 1].kind <= 1 && pc[np - 1].cx == cx && pc[np - 1].cy == cy) {
      pc[np - 1].t1 = v;
      continue;
    }
    if (np < ALT_MAXPIECES) {
      pc[np].cx = cx;
      pc[np].cy = cy;
      pc[np].t0 = u;
      pc[np].t1 = v;
      pc[np].kind = 0;
      pc[np].acx = cx;
      pc[np].acy = cy;
      np++;
    }
  }
  /* Pieces near the ends of [ta, tb] become optional. */
  for (int k = 0; k < np; ++k) {
    double a0 = pc[k].t0 > ta ? pc[k].t0 : ta;
    double a1 = pc[k].t1 < tb ? pc[k].t1 : tb;
    double ov = a1 - a0;
    if (pc[k].kind >= 2) {
      if (ov <= -w) pc[k].kind = 4; /* outside */
      continue;
    }
    if (ov > w) pc[k].kind = 0;
    else if (w > 0.0 && ov > -w) pc[k].kind = 1;
    else pc[k].kind = 4;
  }
  return np;
}

static int cell_ok(const ray_t* r, int m, const cand_t* parent, int cx, int cy) {
  const or_ctx* c = r->s->c;
  if (cx < 0 || cy < 0 || cx >= c->w[m] || cy >= c->h[m]) return 0;
  if (parent && (cx / 2 != parent->cx || cy / 2 != parent->cy)) return 0;
  return 1;
}

/* Every candidate list the walk of [ta, tb] at level m may produce. */
static int candidate_variants(alt_t* A, int m, double ta, double tb, const cand_t* parent,
                              cand_t lists[][OR_MAXCAND], int* counts) {
  const ray_t* r = A->r;
  double w = eps_t(A, tb) * r->s->delta;
  piece_t pc[ALT_MAXPIECES];
  int np = build_pieces(r, m, ta, tb, w, pc);
  int amb[ALT_MAXPIECES], nopt[ALT_MAXPIECES], na = 0;
  for (int k = 0; k < np; ++k) {
    if (pc[k].kind == 1) {
      amb[na] = k;
      nopt[na++] = 2;
    } else if (pc[k].kind == 2 || pc[k].kind == 3) {
      amb[na] = k;
      nopt[na++] = 3;
    }
  }
  int nv = 0;
  int sel[ALT_MAXPIECES];
  memset(sel, 0, sizeof(sel));
  for (;;) {
    cand_t* L = lists[nv];
    int n = 0;
    for (int k = 0; k < np; ++k) {
      int kind = pc[k].kind;
      if (kind == 4) continue;
      int cx = pc[k].cx, cy = pc[k].cy;
      if (kind != 0) {
        int o = 0;
        for (int q = 0; q < na; ++q)
          if (amb[q] == k) o = sel[q];
        if (kind == 1 && o == 1) continue;          /* optional piece left out */
        if (kind == 2 && o == 2) continue;          /* corner skipped */
        if (kind == 3 && o == 0) continue;          /* corner absent nominally */
        if ((kind == 2 && o == 1) || (kind == 3 && o == 2)) {
          cx = pc[k].acx;
          cy = pc[k].acy;
        }
      }
      if (!cell_ok(r, m, parent, cx, cy)) continue;
      double t0 = pc[k].t0 < ta ? ta : (pc[k].t0 > tb ? tb : pc[k].t0);
      double t1 = pc[k].t1 < ta ? ta : (pc[k].t1 > tb ? tb : pc[k].t1);
      if (n > 0 && L[n - 1].cx == cx && L[n - 1].cy == cy) {
        L[n - 1].t_out = t1;
        continue;
      }
      if (n < OR_MAXCAND) {
        L[n].cx = cx;
        L[n].cy = cy;
        L[n].t_in = t0;
        L[n].t_out = t1;
        n++;
      }
    }
    /* keep distinct lists only */
    int dup = 0;
    for (int v = 0; v < nv && !dup; ++v) {
      if (counts[v] != n) continue;
      int same = 1;
      for (int k = 0; k < n && same; ++k)
        same = lists[v][k].cx == L[k].cx && lists[v][k].cy == L[k].cy &&
               lists[v][k].t_in == L[k].t_in && lists[v][k].t_out == L[k].t_out;
      dup = same;
    }
    if (!dup) {
      counts[nv] = n;
      nv++;
      if (nv >= ALT_MAXVARIANTS) {
        A->overflow = 1;
        return nv;
      }
    }
    int q = 0;
    while (q < na) {
      sel[q]++;
      if (sel[q] < nopt[q]) break;
      sel[q] = 0;
      q++;
    }
    if (q >= na) break;
  }
  return nv;
}

static void final_alternatives(alt_t* A, const cand_t* base, valset* out) {
  const ray_t* r = A->r;
  const setup_t* s = r->s;
  double tmid = 0.5 * (base->t_in + base->t_out);
  double arg = (tmid - s->tau0) / (0.5 * s->delta) + 0.5;
  double ea = 2.0 * eps_t(A, tmid);
  long ncs[3];
  int nnc = 0;
  long nc = (long)floor(arg);
  ncs[nnc++] = nc;
  if (ea > 0.0 && arg - floor(arg) < ea) ncs[nnc++] = nc - 1;
  if (ea > 0.0 && floor(arg) + 1.0 - arg < ea) ncs[nnc++] = nc + 1;
  for (int a = 0; a < nnc; ++a) {
    long c0 = ncs[a];
    double dh[3];
    long nn[3];
    int st[3]; /* 0 invalid, 1 valid, 2 optional */
    for (int q = 0; q < 3; ++q) {
      nn[q] = c0 + 1 - q; /* far first */
      st[q] = 0;
      dh[q] = INFINITY;
      if (nn[q] < 0) continue;
      double t = or_t_grid(s, nn[q]);
      double qx, qy, Ht;
      or_ray_point(r, t, &qx, &qy, &Ht);
      double W = s->p->width, H = s->p->rows;
      double e = eps_t(A, t);
      int in = or_inside(s, qx, qy);
      double dmin = fmin(fmin(qx, W - qx), fmin(qy, H - qy));
      if (fabs(dmin) < e) st[q] = 2;
      else st[q] = in ? 1 : 0;
      if (st[q] != 0) {
        /* a sample just outside is evaluated at the clamped edge if taken */
        dh[q] = Ht - or_bilinear(s, qx < 0 ? 0 : (qx >= W ? W - 1e-9 : qx),
                                 qy < 0 ? 0 : (qy >= H ? H - 1e-9 : qy));
      }
    }
    for (int mask = 0; mask < 8; ++mask) {
      int ok = 1;
      for (int q = 0; q < 3; ++q) {
        int bit = (mask >> q) & 1;
        if (st[q] == 0 && bit) ok = 0;
        if (st[q] == 1 && !bit) ok = 0;
      }
      if (!ok) continue;
      if (--A->budget < 0) {
        A->overflow = 1;
        return;
      }
      double best = INFINITY;
      for (int q = 0; q < 3; ++q)
        if ((mask >> q) & 1 && dh[q] < best) best = dh[q];
      if (!isfinite(best)) {
        vs_add(A, out, INFINITY);
        continue;
      }
      for (int q = 0; q < 3; ++q) {
        if (!((mask >> q) & 1)) continue;
        double tq = or_t_grid(s, nn[q]);
        if (dh[q] <= best + eps_h(A, tq)) {
          vs_add(A, out, or_alpha_of(r, tq, dh[q]));
          if (eps_h(A, tq) == 0.0) break; /* exact ties keep the farther sample */
        }
      }
    }
  }
}

static void descend(alt_t* A, int m, const cand_t* cands, int n, valset* out) {
  if (A->overflow) return;
  if (--A->budget < 0) {
    A->overflow = 1;
    return;
  }
  double lb[OR_MAXCAND];
  double best = INFINITY;
  for (int k = 0; k < n; ++k) {
    lb[k] = or_lower_bound(A->r, m, &cands[k]);
    if (lb[k] < best) best = lb[k];
  }
  if (n == 0) return;
  for (int k = n - 1; k >= 0; --k) {
    double e = eps_h(A, cands[k].t_out);
    int take = e > 0.0 ? lb[k] <= best + e : lb[k] == best;
    if (!take) continue;
    if (e == 0.0) {
      /* exact ties keep the farther texel: only the last minimum counts */
      int later = 0;
      for (int q = k + 1; q < n; ++q)
        if (lb[q] == best) later = 1;
      if (later) continue;
    }
    if (m == 0) {
      final_alternatives(A, &cands[k], out);
      continue;
    }
    cand_t lists[ALT_MAXVARIANTS][OR_MAXCAND];
    int counts[ALT_MAXVARIANTS];
    int nv = candidate_variants(A, m - 1, cands[k].t_in, cands[k].t_out, &cands[k], lists, counts);
    for (int v = 0; v < nv; ++v)
      if (counts[v] > 0) descend(A, m - 1, lists[v], counts[v], out);
    if (A->overflow) return;
  }
}

static void segment_alternatives(alt_t* A, int jseg, valset* out) {
  const ray_t* r = A->r;
  const setup_t* s = r->s;
  double ta = s->tau[jseg];
  double w = eps_t(A, ta) * s->delta;
  double tb = ta + ldexp(s->delta, s->m0[jseg]);
  if (r->texit - ta < w) vs_add(A, out, INFINITY);
  if (!(ta < r->texit + w)) return;
  if (tb > r->texit) tb = r->texit;
  if (tb < ta) tb = ta;
  int m = s->m0[jseg];
  cand_t lists[ALT_MAXVARIANTS][OR_MAXCAND];
  int counts[ALT_MAXVARIANTS];
  int nv = candidate_variants(A, m, ta, tb, NULL, lists, counts);
  for (int v = 0; v < nv; ++v) {
    if (counts[v] == 0) {
      vs_add(A, out, INFINITY);
      continue;
    }
    descend(A, m, lists[v], counts[v], out);
  }
}

/* Uniform stepping (Sec. 2, Fig. 1b; Sec. 6.3) takes one kind of discrete
 * decision: which steps count, i.e. lie inside the tile and within the cap.
 * A step whose position is within the position tolerance of the tile edge, or
 * whose length is within it of the cap, may count or not (a step just outside
 * is evaluated at the clamped edge if taken); every other step counts exactly
 * as in the plain loop.  The minimum over the steps that surely count is a
 * valid result, and so is each optional step's clearance below it (a subset of
 * the optional steps yields the smallest of them, or the sure minimum). */
static void uniform_alternatives(alt_t* A, double du, valset* out) {
  const ray_t* r = A->r;
  const setup_t* s = r->s;
  const double W = s->p->width, H = s->p->rows;
  double sure = INFINITY;
  valset opt;
  opt.n = 0;
  for (long k = 0;; ++k) {
    if (--A->budget < 0) {
      A->overflow = 1;
      return;
    }
    const double t = s->tau0 + (double)k * du;
    const double e = eps_t(A, t);
    const double ecap = e * s->delta;
    double qx, qy, Ht;
    or_ray_point(r, t, &qx, &qy, &Ht);
    const double dmin = fmin(fmin(qx, W - qx), fmin(qy, H - qy));
    const int cap_opt = ecap > 0.0 && fabs(t - s->tcap_uniform) <= ecap;
    const int edge_opt = e > 0.0 && fabs(dmin) < e;
    if (t > s->tcap_uniform && !cap_opt) break;
    if (!or_inside(s, qx, qy) && !edge_opt) break;
    const double dh = Ht - or_bilinear(s, qx < 0 ? 0 : (qx >= W ? W - 1e-9 : qx),
                                       qy < 0 ? 0 : (qy >= H ? H - 1e-9 : qy));
    const double a = or_alpha_of(r, t, dh);
    if (cap_opt || edge_opt)
      vs_add(A, &opt, a);
    else if (a < sure)
      sure = a;
  }
  vs_add(A, out, sure);
  for (int k = 0; k < opt.n; ++k)
    if (opt.v[k] < sure) vs_add(A, out, opt.v[k]);
}

int32_t or_alternatives(const or_ctx* c, const or_params* p, int64_t ray, double eh_abs,
                        double eh_rel, double et_abs, double et_rel, double* alpha_out,
                        int32_t max_out) {
  if (!c || !p || p->mode < 0 || p->mode > 2) return -2;
  if (ray < 0 || ray >= (int64_t)c->W * c->H) return -2;
  setup_t s;
  or_setup(&s, c, p);
  ray_t r;
  or_ray_init(&r, &s, (int)(ray % c->W), (int)(ray / c->W));
  alt_t A;
  A.r = &r;
  A.eh_abs = eh_abs;
  A.eh_rel = eh_rel;
  A.et_abs = et_abs;
  A.et_rel = et_rel;
  A.budget = 200000;
  A.overflow = 0;
  if (p->mode != 0) {
    /* uniform stepping (mode 1) and the exact mode, defined as the minimum over
     * the half-texel grid (mode 2) */
    valset res;
    res.n = 0;
    A.budget = 4000000;
    uniform_alternatives(&A, p->mode == 1 ? p->uniform_step * s.delta : 0.5 * s.delta, &res);
    if (A.overflow) return -1;
    int n = res.n < max_out ? res.n : max_out;
    for (int k = 0; k < n; ++k) alpha_out[k] = res.v[k];
    return n;
  }
  static __thread valset segs[OR_MAXSEG];
  for (int j = 0; j < s.nseg; ++j) {
    segs[j].n = 0;
    segment_alternatives(&A, j, &segs[j]);
    if (A.overflow) return -1;
    if (segs[j].n == 0) vs_add(&A, &segs[j], INFINITY);
  }
  /* v is a possible minimum when it is possible for its own segment and every
   * other segment can yield something no smaller. */
  valset res;
  res.n = 0;
  for (int j = 0; j < s.nseg; ++j) {
    for (int k = 0; k < segs[j].n; ++k) {
      double v = segs[j].v[k];
      int ok = 1;
      for (int q = 0; q < s.nseg && ok; ++q) {
        if (q == j) continue;
        double mx = -INFINITY;
        for (int z = 0; z < segs[q].n; ++z)
          if (segs[q].v[z] > mx) mx = segs[q].v[z];
        if (mx < v) ok = 0;
      }
      if (ok) vs_add(&A, &res, v);
    }
  }
  if (s.nseg == 0) vs_add(&A, &res, INFINITY);
  if (A.overflow) return -1;
  int n = res.n < max_out ? res.n : max_out;
  for (int k = 0; k < n; ++k) alpha_out[k] = res.v[k];
  return n;
}
