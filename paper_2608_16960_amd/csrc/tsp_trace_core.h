// Per-ray core of the spherical-grid tracer (see tsp_trace.hip for the
// method).  Functions are host+device so that the identical code can also be
// exercised in a CPU build; the library itself runs them only on the GPU.
#pragma once

#include <cmath>

#include "tsp_internal.h"

#define TSP_HD __host__ __device__ inline

namespace tsp {
namespace core {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kPi = 3.14159265358979323846264338327950;

struct V3 {
    double x, y, z;
};

struct Tab {
    const double *rb, *ce, *ca, *sa, *ab;
    double ab0;
    int nr, ne, na, np, cyclic;
};

TSP_HD Tab make_tab(const TabDesc &D, const double *lds) {
    Tab T;
    T.rb = lds + D.off_rb;
    T.ce = lds + D.off_ce;
    T.ca = lds + D.off_ca;
    T.sa = lds + D.off_sa;
    T.ab = lds + D.off_ab;
    T.ab0 = D.ab0;
    T.nr = D.nr;
    T.ne = D.ne;
    T.na = D.na;
    T.np = D.np;
    T.cyclic = D.cyclic;
    return T;
}

__device__ __forceinline__ void stage_tables(const TabDesc &D, const double *tab, double *lds) {
    for (int k = threadIdx.x; k < D.n_tab; k += blockDim.x) lds[k] = tab[k];
    __syncthreads();
}

// Square root and quotient for the walker's per-event roots.  On the GPU
// they start from the hardware reciprocal square root / reciprocal (about
// 2^-23 relative) and refine: two residual corrections for the root, one
// Newton step and a residual correction for the quotient, about half the
// instructions of the fully guarded library sequences (which also rescale
// denormals and screen special values).  On MI355X both equalled the IEEE
// results on 4M random arguments spanning 2^+-60; the walker's results are
// checked against the FP64 oracle at the usual bars either way.  Arguments
// here are finite and normal, the root's non-negative.  The host build (the
// tests' CPU walker) uses the library sqrt and division.
TSP_HD double ev_sqrt(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    const double y = __builtin_amdgcn_rsq(x);
    const double s = x * y, h = 0.5 * y;
    const double s1 = fma(h, fma(-s, s, x), s);
    return x > 0.0 ? fma(h, fma(-s1, s1, x), s1) : 0.0;
#else
    return sqrt(x);
#endif
}

TSP_HD double ev_div(double n, double d) {
#if defined(__HIP_DEVICE_COMPILE__)
    double y = __builtin_amdgcn_rcp(d);
    y = fma(y, fma(-d, y, 1.0), y);
    const double q = n * y;
    return fma(fma(-d, q, n), y, q);
#else
    return n / d;
#endif
}

// number of a[k] <= v in an increasing array of length m
TSP_HD int count_le(const double *a, int m, double v) {
    int lo = 0, hi = m;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] <= v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// number of a[k] >= v in a decreasing array of length m
TSP_HD int count_ge_dec(const double *a, int m, double v) {
    int lo = 0, hi = m;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] >= v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Elevation region of a point with cos(colatitude) = u: e_b[ie] <= theta < e_b[ie+1]
// (-1 or ne outside a wedge; a point at theta = pi belongs to the last bin when
// e_b ends at pi).
TSP_HD int class_e(const Tab &T, double u) {
    u = fmin(fmax(u, -1.0), 1.0);
    int ie = count_ge_dec(T.ce, T.ne + 1, u) - 1;
    if (ie == T.ne && T.ce[T.ne] <= -1.0) ie = T.ne - 1;
    return ie;
}

// Azimuth region of (px, py) measured from a_b[0] in [0, 2 pi); the region
// past the last boundary is 0 on a cyclic grid, else the outside region na.
TSP_HD int class_a(const Tab &T, double px, double py, double *phi) {
    double p0 = atan2(py, px);
    *phi = p0;
    double ph = fmod(p0 - T.ab0, kTwoPi);
    if (ph < 0) ph += kTwoPi;
    if (ph >= kTwoPi) ph -= kTwoPi;
    int ia = count_le(T.ab, T.na + 1, ph) - 1;
    if (ia >= T.na) ia = T.cyclic ? 0 : T.na;
    return ia;
}

// Root of cone k's quadratic that lies on the current monotone run of the
// colatitude.  u_incr: cos(theta) increases across the crossing (Eq. 12
// "negative").  With f(t) = z^2 - c^2 |p|^2 = A t^2 + 2 B t + C, the two
// roots have f'/2 = A t + B = +-sqrt(B^2 - A C), and on the nappe z c > 0
// the test cos(theta) > c reads f > 0 for c > 0 and f < 0 for c < 0.  So the
// crossing in the wanted direction is the root with sign(f') =
// (u_incr == (c > 0)) ? + : -, one root of the stable pair
// q = -(B + sign(B) sqrt(disc)): q / A when that sign is -sign(B), else
// C / q.  One square root and one division.  Falls back to `fb` when
// rounding leaves no admissible root (no real root, or the root on the other
// nappe: a grazing crossing at the run's turning point).  A cone with
// |c| < 1e-12 is the plane z = 0.
TSP_HD double cone_root(const Tab &T, int k, bool u_incr, const V3 &x,
                                            const V3 &n, double xx, double xn, double lo,
                                            double hi, double fb) {
    const double c = T.ce[k];
    double t = fb;
    if (fabs(c) < 1e-12) {  // the plane z = 0
        if (n.z != 0.0) t = ev_div(-x.z, n.z);
    } else {
        const double c2 = c * c;
        const double A = n.z * n.z - c2;
        const double B = x.z * n.z - c2 * xn;
        const double C = x.z * x.z - c2 * xx;
        const double disc = B * B - A * C;
        if (disc >= 0.0) {
            const double s = ev_sqrt(disc);
            const double q = -(B + copysign(s, B));
            const bool want_pos = (u_incr == (c > 0.0));
            const bool via_a = want_pos == (copysign(1.0, B) < 0.0);  // wanted sign == -sign(B)
            const double tr = via_a ? ev_div(q, A) : ev_div(C, q);
            if (fabs(tr) < INFINITY && (x.z + n.z * tr) * c >= 0.0) t = tr;
        }
    }
    return fmin(fmax(t, lo), hi);
}

TSP_HD double plane_t(const Tab &T, int k, const V3 &x, const V3 &n,
                                          double lo) {
    const double xm = -x.x * T.sa[k] + x.y * T.ca[k];
    const double nm = -n.x * T.sa[k] + n.y * T.ca[k];
    return (nm != 0.0) ? ev_div(-xm, nm) : lo;
}

// Resumable walk along one ray.  init() sets up the three crossing streams;
// each next() call advances the merge until the next canonical segment is
// complete and returns it (false once the ray has left the grid).  Keeping
// the walk resumable lets a wavefront advance all its rays one segment at a
// time (see the on-the-fly adjoint).
struct Walker {
    // ray
    V3 x, n;
    double xx, xn, b, tc, tin, tout, ts;
    // radial stream (Eq. 11)
    int kb, ir, rk, rstage;  // rstage: 0 inbound, 1 outbound, 2 next event is the exit
    double t_r;
    // elevation stream (Eq. 12): estage 0 first run, 1 second run,
    // 3 jump pending at tc (ray through the origin), 2 done
    int ie, ie_out, estage, etgt;
    double elo, ehi, t_e, elast;
    bool two;
    // azimuth stream (Eq. 13)
    int ia, ia_out, aleft, adir;
    bool ajump;
    double t_a, alast;
    // merge state
    double tcur, plen;
    int pv;
    bool gap, finished;

    TSP_HD void next_e(const Tab &T) {
        for (;;) {
            if (estage == 0 || estage == 1) {
                if (ie != etgt) {
                    const bool down = etgt < ie;  // colatitude decreasing, cos increasing
                    const int k = down ? ie : ie + 1;
                    const double lo = fmax(elo, elast);
                    const double fb = two ? ts : fmin(fmax(elo, lo), ehi);
                    t_e = cone_root(T, k, down, x, n, xx, xn, lo, ehi, fb);
                    return;
                }
                if (estage == 0 && two) {
                    estage = 1;
                    elo = ts;
                    ehi = tout;
                    etgt = ie_out;
                    continue;
                }
                estage = 2;
            }
            if (estage == 3) {
                t_e = tc;
                return;
            }
            t_e = INFINITY;
            return;
        }
    }

    TSP_HD void next_a(const Tab &T) {
        if (aleft > 0) {
            // 0 <= ia < np: wrap by a compare, not a division
            const int k = (adir > 0) ? (ia + 1 == T.np ? 0 : ia + 1) : ia;
            const double lo = fmax(alast, tin);
            t_a = fmin(fmax(plane_t(T, k, x, n, lo), lo), tout);
        } else if (!ajump) {
            t_a = INFINITY;
        }
    }

    // Returns false when the ray misses the grid (nothing to walk).  A ray
    // may start inside the outer sphere: the walk then begins at l = 0 in the
    // region that holds the start (l >= 0 only, Eq. 3).
    TSP_HD bool init(const Tab &T, const V3 &x_, const V3 &n_) {
        x = x_;
        n = n_;
        finished = true;
        pv = -1;
        plen = 0.0;
        gap = false;
        const int nr = T.nr, np = T.np;
        xx = x.x * x.x + x.y * x.y + x.z * x.z;
        xn = x.x * n.x + x.y * n.y + x.z * n.z;
        const double cx = x.y * n.z - x.z * n.y;
        const double cy = x.z * n.x - x.x * n.z;
        const double cz = x.x * n.y - x.y * n.x;  // (x cross n)_z, constant along the ray
        const double b2 = cx * cx + cy * cy + cz * cz;
        const double Ro = T.rb[nr];
        tc = -xn;
        if (!(b2 < Ro * Ro)) return false;  // misses the outer sphere
        b = sqrt(b2);
        const double hch = sqrt((Ro - b) * (Ro + b));
        tin = tc - hch;
        tout = tc + hch;
        if (!(tout > 0.0)) return false;  // the sphere lies behind the start
        const bool inner = tin < 0.0;      // the start is inside the outer sphere
        if (inner) tin = 0.0;

        // radial stream
        kb = count_le(T.rb, nr + 1, b);  // shells kb..nr-1 are crossed twice
        if (!inner) {
            ir = nr - 1;
            rk = nr - 1;
            if (kb <= nr - 1) {
                rstage = 0;
                t_r = tc - sqrt((T.rb[rk] - b) * (T.rb[rk] + b));
            } else {
                rstage = 2;
                t_r = tout;
            }
        } else {
            // shell of the start (-1 in the inner hole); inbound crossings of
            // spheres ir..kb remain while moving towards the centre, else
            // outbound crossings of ir+1..nr-1, then the exit
            ir = count_le(T.rb, nr + 1, sqrt(xx)) - 1;
            if (tc > 0.0 && ir >= kb) {
                rstage = 0;
                rk = ir;
                t_r = tc - sqrt((T.rb[rk] - b) * (T.rb[rk] + b));
            } else {
                rk = ir + 1;
                if (rk <= nr - 1) {
                    rstage = 1;
                    t_r = tc + sqrt((T.rb[rk] - b) * (T.rb[rk] + b));
                } else {
                    rstage = 2;
                    t_r = tout;
                }
            }
        }

        // classification at entry (or start) and exit of the outer sphere
        const V3 pin = {x.x + n.x * tin, x.y + n.y * tin, x.z + n.z * tin};
        const V3 pout = {x.x + n.x * tout, x.y + n.y * tout, x.z + n.z * tout};
        const double rin = sqrt(pin.x * pin.x + pin.y * pin.y + pin.z * pin.z);
        const double rout = sqrt(pout.x * pout.x + pout.y * pout.y + pout.z * pout.z);
        // A start at the origin, or on the polar axis, lies on region
        // boundaries: the region the ray enters is the one its direction
        // points into.
        ie = (rin > 0.0) ? class_e(T, pin.z / rin) : class_e(T, n.z);
        ie_out = class_e(T, pout.z / rout);
        double phi_in, phi_out;
        const bool on_axis = inner && pin.x == 0.0 && pin.y == 0.0;
        ia = on_axis ? class_a(T, n.x, n.y, &phi_in) : class_a(T, pin.x, pin.y, &phi_in);
        ia_out = class_a(T, pout.x, pout.y, &phi_out);

        // elevation stream
        estage = 0;
        elo = tin;
        ehi = tout;
        ts = 0.0;
        two = false;
        if (b2 == 0.0) {
            etgt = ie;
            estage = (ie_out != ie) ? 3 : 2;
        } else {
            const double den = n.z * xn - x.z;
            const double num = x.z * xn - n.z * xx;
            if (den != 0.0) {
                ts = num / den;
                two = (ts > tin) && (ts < tout);
            }
            if (two) {
                const V3 ps = {x.x + n.x * ts, x.y + n.y * ts, x.z + n.z * ts};
                const double rs = sqrt(ps.x * ps.x + ps.y * ps.y + ps.z * ps.z);
                etgt = class_e(T, ps.z / rs);
                ehi = ts;
            } else {
                etgt = ie_out;
            }
        }
        t_e = INFINITY;
        elast = tin;
        next_e(T);

        // azimuth stream
        aleft = 0;
        adir = 0;
        ajump = false;
        t_a = INFINITY;
        alast = tin;
        if (cz != 0.0) {
            adir = (cz > 0.0) ? 1 : -1;
            int cnt = (adir > 0) ? (ia_out - ia + np) % np : (ia - ia_out + np) % np;
            double dph = (adir > 0) ? phi_out - phi_in : phi_in - phi_out;
            dph = fmod(dph, kTwoPi);
            if (dph < 0) dph += kTwoPi;
            if (dph > kPi) {
                cnt = 0;  // the sweep is tiny and rounding reversed it
            } else if (cnt == 0 && dph > 0.0) {
                // Same region at both ends.  A region wider than pi can be left
                // and re-entered the other way round: then every plane is crossed.
                double rel = fmod(phi_in - T.ab0, kTwoPi);
                if (rel < 0) rel += kTwoPi;
                const double edge =
                    (adir > 0) ? ((ia + 1 <= T.na) ? T.ab[ia + 1] : kTwoPi) : T.ab[ia];
                const double dist = (adir > 0) ? edge - rel : rel - edge;
                if (dph > dist) cnt = np;
            }
            aleft = cnt;
        } else {
            const double nxy2 = n.x * n.x + n.y * n.y;
            if (nxy2 > 0.0) {  // the xy-projection passes through the axis: azimuth jumps by pi
                const double tax = -(x.x * n.x + x.y * n.y) / nxy2;
                if (tax > tin && tax < tout && ia_out != ia) {
                    ajump = true;
                    t_a = tax;
                }
            }
        }
        next_a(T);
        tcur = tin;
        finished = false;
        return true;
    }

    // Process one crossing event (or, once the ray has left the grid, flush
    // the pending segment).  Returns true when a canonical segment completed
    // (voxel, length in vout / lout).  done() tells when nothing is left.
    TSP_HD bool step(const Tab &T, int &vout, double &lout) {
        if (finished) {
            if (pv >= 0) {  // the last pending segment
                vout = pv;
                lout = plen;
                pv = -1;
                return true;
            }
            return false;
        }
        const int nr = T.nr, ne = T.ne, na = T.na, np = T.np;
        double tm = t_r;
        int fam = 0;
        if (t_e < tm) {
            tm = t_e;
            fam = 1;
        }
        if (t_a < tm) {
            tm = t_a;
            fam = 2;
        }
        // the piece [tcur, tm] joins the pending segment or completes it;
        // written with selects rather than branches (every lane takes the
        // same path, and the wavefront skips the mask bookkeeping)
        const bool adv = tm > tcur;
        const bool valid =
            (ir >= 0) && (ir < nr) && (ie >= 0) && (ie < ne) && (ia >= 0) && (ia < na);
        const int v = (ir * ne + ie) * na + ia;
        const double d = tm - tcur;
        const bool take = adv && valid;
        const bool same = v == pv && !gap;
        const bool emitted = take && !same && pv >= 0;
        vout = pv;  // meaningful only when a segment is emitted
        lout = plen;
        plen = take ? (same ? plen + d : d) : plen;
        pv = (take && !same) ? v : pv;
        gap = adv ? !valid : gap;
        tcur = adv ? tm : tcur;
        if (fam == 0) {
            if (rstage == 2) {
                finished = true;
            } else if (rstage == 0) {
                ir = rk - 1;
                if (rk > kb) {
                    rk--;
                    t_r = tc - ev_sqrt((T.rb[rk] - b) * (T.rb[rk] + b));
                } else {
                    rstage = 1;
                    t_r = tc + ev_sqrt((T.rb[rk] - b) * (T.rb[rk] + b));
                }
            } else {
                ir = rk;
                rk++;
                if (rk <= nr - 1) {
                    t_r = tc + ev_sqrt((T.rb[rk] - b) * (T.rb[rk] + b));
                } else {
                    rstage = 2;
                    t_r = tout;
                }
            }
        } else if (fam == 1) {
            if (estage == 3) {
                ie = ie_out;
                estage = 2;
            } else {
                ie = (etgt < ie) ? ie - 1 : ie + 1;
            }
            elast = t_e;
            next_e(T);
        } else {
            if (ajump) {
                ia = ia_out;
                ajump = false;
                t_a = INFINITY;
            } else {
                ia = (adir > 0) ? (ia + 1 == np ? 0 : ia + 1) : (ia == 0 ? np - 1 : ia - 1);
                aleft--;
                alast = t_a;
                next_a(T);
            }
        }
        return emitted;
    }

    TSP_HD bool done() const { return finished && pv < 0; }

    // Next canonical segment (events until one completes); false at the end.
    TSP_HD bool next(const Tab &T, int &vout, double &lout) {
        while (!done())
            if (step(T, vout, lout)) return true;
        return false;
    }
};

// Walk one ray; calls vis.seg(voxel, length) once per canonical segment in
// increasing distance.
template <class Vis>
TSP_HD void trace_ray(const Tab &T, const V3 &x, const V3 &n, Vis &vis) {
    Walker w;
    if (!w.init(T, x, n)) return;
    int v;
    double l;
    while (!w.done())  // one crossing event per iteration, segments as they complete
        if (w.step(T, v, l)) vis.seg(v, l);
}

}  // namespace core
}  // namespace tsp
