// lbm_bc.hpp -- wet-node boundary conditions (Sec. 3.4) for the two-pass scheme.
//
// A boundary node is a fluid cell whose outward neighbour along each of its normals is solid.
// On a face (one normal n) the inward neighbour x_f = x_b - n is a bulk fluid cell; a velocity
// node may also sit on an edge or corner (two or three normals), with bulk fluid cells at
// x_b + d and x_b + 2d along the inward diagonal d = -(sum of the normals), and x_f = x_b + d.
// Its post-advection populations split into P- (incoming through a face: c_i . n_k < 0 for some
// normal, unknown), P0 (c_i . n = 0) and P+ (c_i . n > 0), eq. (bc_rho_components_def).  Three
// node types:
//   velocity node: v_b prescribed; rho_b from mass continuity (bc_density_impermWall) on faces
//                  and extrapolated from the bulk on edges and corners (Sec. 3.4.1, remedy (i)),
//                  or from bounce-back (bc_density_BounceBack) everywhere; populations rebuilt
//                  by the run's scheme;
//   pressure node: one normal; rho_b prescribed, tangential velocity 0, normal velocity from the
//                  same continuity relation; populations rebuilt by the run's scheme;
//   outflow node:  one normal; P- populations copied from x_f (f_bar_outflow_BC).
// Per step: outflow copies -> bulk moments -> boundary records (rho_b, v_b) in two stages ->
// velocity correction -> records fixed to (rho_b, v_b) -> population rebuild -> collide-stream.
// The node kernels run one thread per boundary node.  A node's populations are read from, and
// rebuilt into, the slots its own bulk update reads (each slot is read by exactly one cell), so
// the rebuild touches no other cell's state; NEEM and the outflow copy read x_f's slots, which
// no boundary kernel writes.
#pragma once

#include "lbm_device.hpp"

namespace lbm {

enum : uint32_t { kNodeVelocity = 1, kNodePressure = 2, kNodeOutflow = 3 };

// One boundary node: cell index, type | normal << 8, and the prescribed (v_x, v_y, v_z, rho).
template <typename T>
struct BNodes {
    const uint32_t *cell;
    const uint32_t *code;
    const P4<T> *val;
    uint32_t count;
};

// Outward normal(s) of a node from bits 8..15 of its code: 0..5 for one normal (-x, +x, -y, +y,
// -z, +z), or 64 + ax + 4 ay + 16 az with a = 1 (minus), 2 (plus), 0 (none) for an edge or
// corner.  Returns the number of normals.
__device__ __forceinline__ int normal_of(uint32_t code, int nv[3]) {
    const int k = (int)((code >> 8) & 0xffu);
    nv[0] = nv[1] = nv[2] = 0;
    if (k >= 64) {
        int cnt = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int sa = ((k - 64) >> (2 * a)) & 3;
            nv[a] = sa == 1 ? -1 : (sa == 2 ? 1 : 0);
            cnt += nv[a] != 0 ? 1 : 0;
        }
        return cnt;
    }
    nv[k >> 1] = (k & 1) ? 1 : -1;
    return 1;
}

template <int D, int I>
__device__ __forceinline__ int c_dot(const int nv[3]) {
    using L = Lat<D>;
    return L::c[I][0] * nv[0] + L::c[I][1] * nv[1] + L::c[I][2] * nv[2];
}

// Is f_I one of the unknown incoming populations (P-)?  It points inwards along a normal axis.
template <int D, int I>
__device__ __forceinline__ bool in_pminus(const int nv[3]) {
    using L = Lat<D>;
    return (nv[0] != 0 && L::c[I][0] == -nv[0]) || (nv[1] != 0 && L::c[I][1] == -nv[1]) ||
           (nv[2] != 0 && L::c[I][2] == -nv[2]);
}

__device__ __forceinline__ uint32_t cell_at(const Grid &g, int x, int y, int z) {
    return (uint32_t)x + (uint32_t)g.nx * ((uint32_t)y + (uint32_t)g.ny * (uint32_t)z);
}

__device__ __forceinline__ void cell_xyz(const Grid &g, uint32_t n, int &x, int &y, int &z) {
    x = (int)(n % (uint32_t)g.nx);
    y = (int)((n / (uint32_t)g.nx) % (uint32_t)g.ny);
    z = (int)(n / ((uint32_t)g.nx * (uint32_t)g.ny));
}

// Slot from which cell n reads f_I (the address load_raw uses), for writing rebuilt values.
template <int D, bool SOLIDS, int PH, int I, typename P>
__device__ __forceinline__ P *read_slot(P *__restrict__ f, const uint8_t *__restrict__ mask,
                                        const Grid &g, const Nbr<D> &nb) {
    using L = Lat<D>;
    constexpr int cx = L::c[I][0], cy = L::c[I][1], cz = L::c[I][2];
    const uint32_t n = nb.self();
    if constexpr (PH == 0 || (cx == 0 && cy == 0 && cz == 0)) {
        return at(plane(f, I, g.N), n);
    } else {
        const uint32_t s = nb.at(-cx, -cy, -cz);
        if constexpr (SOLIDS) {
            if (mask[s]) return at(plane(f, I, g.N), n);
        }
        return at(plane(f, L::opp[I], g.N), s);
    }
}

// Write value v of f_I into cell n's read slot, encoded as that slot is decoded.
template <int D, bool SOLIDS, int PH, int I, typename T, typename P, typename E>
__device__ __forceinline__ void write_read_slot(P *__restrict__ f,
                                                const uint8_t *__restrict__ mask, const E &ev,
                                                const Phys<T> &ph, const Grid &g,
                                                const Nbr<D> &nb, T v) {
    *read_slot<D, SOLIDS, PH, I>(f, mask, g, nb) =
        encode<D, I, P>(v, load_sigma<D, SOLIDS, I, P>(mask, ev, ph, nb));
}

// Zero-gradient outflow: f_I(x_b) = f_I(x_f) for I in P-.
template <int D, typename T, typename P, bool SOLIDS, int PH>
__global__ __launch_bounds__(256) void k_bc_outflow(P *__restrict__ f,
                                                    const uint8_t *__restrict__ mask,
                                                    const T *__restrict__ eps, BNodes<T> bn,
                                                    Grid g, Phys<T> ph) {
    const uint32_t k = blockIdx.x * 256u + threadIdx.x;
    if (k >= bn.count) return;
    const uint32_t code = bn.code[k];
    if ((code & 0xffu) != kNodeOutflow) return;
    int nv[3];
    normal_of(code, nv);
    int x, y, z;
    cell_xyz(g, bn.cell[k], x, y, z);
    Nbr<D> nb, nf;
    nb.init(g, x, y, z);
    nf.init(g, wrapk(x, -nv[0], g.nx), wrapk(y, -nv[1], g.ny), wrapk(z, -nv[2], g.nz));
    const EpsGlobal<D, T> eb{eps, &nb}, ef{eps, &nf};
    unroll<0, Lat<D>::Q>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        if (in_pminus<D, i>(nv)) {
            const T v = load_pop<D, SOLIDS, PH, i>(f, mask, ef, ph, g, nf);
            write_read_slot<D, SOLIDS, PH, i>(f, mask, eb, ph, g, nb, v);
        }
    });
}

// W_beta of the viscous term of eq. (accel_approx_boundary) at cell (cx, cy, cz), for a node
// with outward normal nv:
//   nu_eff [ (v_beta / eps) (n . grad eps) + (d_beta eps) (n . v) / eps ],
// v from the records (v^(1) on bulk cells, the boundary velocity on boundary nodes).
template <int D, typename T, bool AD, int BETA>
__device__ __forceinline__ T bc_flux(const P4<T> *__restrict__ m1, const T *__restrict__ eps,
                                     const Grid &g, const Phys<T> &ph, int cx, int cy, int cz,
                                     const int nv[3]) {
    Nbr<D> nc;
    nc.init(g, cx, cy, cz);
    const EpsGlobal<D, T> ev{eps, &nc};
    const uint32_t c = nc.self();
    const T e = ev.at(0, 0, 0);
    T ge[3] = {T(0), T(0), T(0)};
    unroll<0, D>([&](auto ia) {
        constexpr int a = decltype(ia)::value;
        ge[a] = eps_gradient<a, AD>(ev, ph, c);
    });
    const P4<T> r = ld(m1, c);
    const T v[3] = {r.y, r.z, r.w};
    T gn = T(0), vn = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        gn = gn + T(nv[a]) * ge[a];
        vn = vn + T(nv[a]) * v[a];
    }
    return viscosity(ph, e).nu * (dv(v[BETA], e) * gn + ge[BETA] * dv(vn, e));
}

// Viscous term of eq. (accel_approx_boundary) at face node (x, y, z): the divergence of W with
// each d/dx_beta by the derivative rule of moment fields (one-sided next to solids).
template <int D, typename T, bool AD>
__device__ __forceinline__ T bc_viscous_term(const P4<T> *__restrict__ m1,
                                             const T *__restrict__ eps,
                                             const uint8_t *__restrict__ mask, const Grid &g,
                                             const Phys<T> &ph, int x, int y, int z,
                                             const int nv[3]) {
    T div = T(0);
    unroll<0, D>([&](auto ib) {
        constexpr int beta = decltype(ib)::value;
        T v5[5];
        bool f5[5];
#pragma unroll
        for (int k = -2; k <= 2; ++k) {
            const int cx = beta == 0 ? wrapk(x, k, g.nx) : x;
            const int cy = beta == 1 ? wrapk(y, k, g.ny) : y;
            const int cz = beta == 2 ? wrapk(z, k, g.nz) : z;
            f5[k + 2] = k == 0 || !mask[cell_at(g, cx, cy, cz)];
            v5[k + 2] = f5[k + 2] ? bc_flux<D, T, AD, beta>(m1, eps, g, ph, cx, cy, cz, nv) : T(0);
        }
        div = div + deriv_rule(v5, f5);
    });
    return div;
}

// Records (rho_b, v_b) of velocity and pressure nodes, written over the bulk moment pass, in
// two stages (one launch each).
// Stage 0, every node:
//   velocity node: bounce-back rule: rho_b = sum of its post-advection populations / eps_b, eq.
//     (bc_density_BounceBack) with halfway bounce-back in the streaming; continuity rule on a
//     face: rho_b = (S0 + 2 S+) / (eps_b + v_perp - a_perp / 2) with a_perp = eps_b b_perp -
//     mu_D v_perp - mu_F |v_b| v_perp + RT d(eps)/dn (eq. accel_approx_boundary without its
//     viscous term); continuity rule on an edge or corner, where the relation does not apply:
//     rho_b = 2 rho(x_b + d) - rho(x_b + 2d) along the inward diagonal d;
//   pressure node: v_perp (1 + mu_D / 2) + (mu_F / 2) |v_perp| v_perp = R,
//     R = (S0 + 2 S+) / rho_b - eps_b + (eps_b b_perp + RT d(eps)/dn) / 2, closed form as v_(1).
// Stage 1, face velocity nodes under the continuity rule: rho_b again with the viscous term in
//   a_perp, from the velocities stage 0 left in the records.  Other threads read only the
//   velocity of a node's record, which this stage rewrites with the same value.
template <int D, typename T, typename P, bool SOLIDS, int PH, bool AD>
__global__ __launch_bounds__(256) void k_bc_records(const P *__restrict__ f,
                                                    const uint8_t *__restrict__ mask,
                                                    const T *__restrict__ eps,
                                                    const T *__restrict__ muD,
                                                    const T *__restrict__ muF,
                                                    P4<T> *__restrict__ m1, BNodes<T> bn, Grid g,
                                                    Phys<T> ph, int bounce_back_density,
                                                    int stage) {
    const uint32_t k = blockIdx.x * 256u + threadIdx.x;
    if (k >= bn.count) return;
    const uint32_t code = bn.code[k];
    const uint32_t type = code & 0xffu;
    if (type != kNodeVelocity && type != kNodePressure) return;
    int nv[3];
    const int nn = normal_of(code, nv);
    if (stage == 1 && (type != kNodeVelocity || nn != 1 || bounce_back_density)) return;
    int x, y, z;
    const uint32_t n = bn.cell[k];
    cell_xyz(g, n, x, y, z);
    Nbr<D> nb;
    nb.init(g, x, y, z);
    const EpsGlobal<D, T> ev{eps, &nb};
    T s0 = T(0), sp = T(0), sum = T(0);
    unroll<0, Lat<D>::Q>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        const T fi = load_pop<D, SOLIDS, PH, i>(f, mask, ev, ph, g, nb);
        sum = sum + fi;
        const int cn = c_dot<D, i>(nv);
        if (cn == 0) s0 = s0 + fi;
        else if (cn > 0) sp = sp + fi;
    });
    const T e = ev.at(0, 0, 0);
    T gperp = T(0), bperp = T(0);
    unroll<0, D>([&](auto ia) {
        constexpr int a = decltype(ia)::value;
        gperp = gperp + T(nv[a]) * eps_gradient<a, AD>(ev, ph, n);
        bperp = bperp + T(nv[a]) * ph.b[a];
    });
    const P4<T> pv = bn.val[k];
    T vb[3] = {pv.x, pv.y, pv.z};
    T rho;
    if (type == kNodeVelocity) {
        T vperp = T(0), s = T(0);
#pragma unroll
        for (int a = 0; a < D; ++a) vperp = vperp + T(nv[a]) * vb[a];
#pragma unroll
        for (int a = 0; a < D; ++a) s = s + vb[a] * vb[a];
        const T vm = sq(s);
        if (bounce_back_density) {
            rho = div_rn(sum, e);
        } else if (nn > 1) {
            const uint32_t f1 = cell_at(g, wrapk(x, -nv[0], g.nx), wrapk(y, -nv[1], g.ny),
                                        wrapk(z, -nv[2], g.nz));
            const uint32_t f2 = cell_at(g, wrapk(x, -2 * nv[0], g.nx),
                                        wrapk(y, -2 * nv[1], g.ny), wrapk(z, -2 * nv[2], g.nz));
            rho = T(2) * ld(m1, f1).x - ld(m1, f2).x;
        } else {
            T aperp = ((e * bperp - ld(muD, n) * vperp) - (ld(muF, n) * vm) * vperp) +
                      ph.RT * gperp;
            if (stage == 1)
                aperp = aperp + bc_viscous_term<D, T, AD>(m1, eps, mask, g, ph, x, y, z, nv);
            rho = dv(s0 + T(2) * sp, (e + vperp) - T(0.5) * aperp);
        }
    } else {
        rho = pv.w;
        const T R = (dv(s0 + T(2) * sp, rho) - e) + T(0.5) * (e * bperp + ph.RT * gperp);
        const T c1 = T(1) + T(0.5) * ld(muD, n), c2 = T(0.5) * ld(muF, n);
        const T vperp = dv(T(2) * R, c1 + sq(c1 * c1 + (T(4) * c2) * (R < T(0) ? -R : R)));
#pragma unroll
        for (int a = 0; a < 3; ++a) vb[a] = T(nv[a]) * vperp;
    }
    *at(m1, n) = pack(rho, vb[0], vb[1], D == 3 ? vb[2] : T(0));
}

// After the velocity correction: the corrected velocity of velocity and pressure nodes is v_b.
template <typename T>
__global__ __launch_bounds__(256) void k_bc_fix(const P4<T> *__restrict__ m1,
                                                P4<T> *__restrict__ m2, BNodes<T> bn) {
    const uint32_t k = blockIdx.x * 256u + threadIdx.x;
    if (k >= bn.count) return;
    const uint32_t type = bn.code[k] & 0xffu;
    if (type != kNodeVelocity && type != kNodePressure) return;
    const uint32_t n = bn.cell[k];
    *at(m2, n) = ld(m1, n);
}

// Equilibrium populations (prod_form) at velocity w: xi = w / eps, P = xi^2 + RT.
template <int D, typename T>
__device__ __forceinline__ void eq_at(T e, T rho, const T w[3], T RT, ProductForm<D, T> &pf) {
    T xi[3] = {T(0), T(0), T(0)}, P[3] = {RT, RT, RT};
#pragma unroll
    for (int a = 0; a < D; ++a) {
        xi[a] = dv(w[a], e);
        P[a] = xi[a] * xi[a] + RT;
    }
    pf.init(e * rho, xi, P);
}

// Acceleration of cell nb from the (rho, v) records: its own from m2, its stencil neighbours'
// from nbr (the same buffer, or the previous step's in a lagged step).
template <int D, typename T, bool SOLIDS, bool AD>
__device__ __forceinline__ void node_accel(const P4<T> *__restrict__ m2,
                                           const P4<T> *__restrict__ nbr,
                                           const T *__restrict__ eps, const T *__restrict__ muD,
                                           const T *__restrict__ muF,
                                           const uint8_t *__restrict__ mask, const Grid &g,
                                           const Phys<T> &ph, const Nbr<D> &nb,
                                           const EpsGlobal<D, T> &ev, Rec<T> &own, Visc<T> &vs,
                                           T acc[3]) {
    own = load_rec<D>(m2, nb.self(), ev.at(0, 0, 0));
    const CellStatic<D, T> cs = cell_static<D, AD>(ev, ph, nb.self(), own.e);
    vs = cs.vs;
    Rec<T> rec[3][2];
    bool fl[3][2];
    load_stencil<D, T, SOLIDS>(nbr, ev, mask, g, nb, rec, fl);
    accel_of<D, T, SOLIDS>(nbr, eps, muD, muF, mask, g, ph, nb, own, rec, fl, cs.ge, cs.H, cs.vs,
                           acc);
}

// Rebuild of all post-advection populations of velocity and pressure nodes, lambda = dt = 1,
// f^tgt = f^eq(eps_b, rho_b, v_b), f^* = f^eq(eps_b, rho_b, v_b + a_b):
//   scheme 0, eq. (eq_bc_f_bar): f_i = (3/2) f^tgt_i - (1/2) f^*_i;
//   scheme 1, eqs. (NEEM_bc_f_bar), (zeta_beta_NEEM):
//     f_i = zeta f_i(x_f) + (3/2)[f^tgt_i - zeta f^eq_i(x_f)] + (1/2)[zeta f^*_i(x_f) - f^*_i];
//   scheme 2, TMS (Sec. 3.4.4, steps 1-3).
template <int D, typename T, typename P, bool SOLIDS, int PH, bool AD>
__global__ __launch_bounds__(256) void k_bc_rebuild(P *__restrict__ f,
                                                    const P4<T> *__restrict__ m2,
                                                    const P4<T> *__restrict__ nbr,
                                                    const T *__restrict__ eps,
                                                    const T *__restrict__ muD,
                                                    const T *__restrict__ muF,
                                                    const uint8_t *__restrict__ mask,
                                                    BNodes<T> bn, Grid g, Phys<T> ph,
                                                    int scheme) {
    using L = Lat<D>;
    const uint32_t k = blockIdx.x * 256u + threadIdx.x;
    if (k >= bn.count) return;
    const uint32_t code = bn.code[k];
    const uint32_t type = code & 0xffu;
    if (type != kNodeVelocity && type != kNodePressure) return;
    int nv[3];
    normal_of(code, nv);
    int x, y, z;
    cell_xyz(g, bn.cell[k], x, y, z);
    Nbr<D> nb;
    nb.init(g, x, y, z);
    const EpsGlobal<D, T> ev{eps, &nb};
    Rec<T> own;
    Visc<T> vs;
    T acc[3];
    node_accel<D, T, SOLIDS, AD>(m2, nbr, eps, muD, muF, mask, g, ph, nb, ev, own, vs, acc);
    T vstar[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int a = 0; a < D; ++a) vstar[a] = own.w[a] + acc[a];
    ProductForm<D, T> ftgt, fst;
    eq_at<D>(own.e, own.r, own.w, ph.RT, ftgt);
    eq_at<D>(own.e, own.r, vstar, ph.RT, fst);
    if (scheme == 0) {
        unroll<0, L::Q>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            const T v = T(1.5) * ftgt.template at<i>() - T(0.5) * fst.template at<i>();
            write_read_slot<D, SOLIDS, PH, i>(f, mask, ev, ph, g, nb, v);
        });
    } else if (scheme == 1) {
        Nbr<D> nf;
        nf.init(g, wrapk(x, -nv[0], g.nx), wrapk(y, -nv[1], g.ny), wrapk(z, -nv[2], g.nz));
        const EpsGlobal<D, T> evf{eps, &nf};
        Rec<T> ownf;
        Visc<T> vsf;
        T accf[3];
        node_accel<D, T, SOLIDS, AD>(m2, nbr, eps, muD, muF, mask, g, ph, nf, evf, ownf, vsf,
                                     accf);
        T vfs[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int a = 0; a < D; ++a) vfs[a] = ownf.w[a] + accf[a];
        ProductForm<D, T> feqf, fstf;
        eq_at<D>(ownf.e, ownf.r, ownf.w, ph.RT, feqf);
        eq_at<D>(ownf.e, ownf.r, vfs, ph.RT, fstf);
        const T zeta = dv(T(1) - vsf.beta, T(1) - vs.beta);
        T fb[L::Q];
        unroll<0, L::Q>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            const T ff = load_pop<D, SOLIDS, PH, i>(f, mask, evf, ph, g, nf);
            fb[i] = (zeta * ff + T(1.5) * (ftgt.template at<i>() - zeta * feqf.template at<i>())) +
                    T(0.5) * (zeta * fstf.template at<i>() - fst.template at<i>());
        });
        unroll<0, L::Q>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            write_read_slot<D, SOLIDS, PH, i>(f, mask, ev, ph, g, nb, fb[i]);
        });
    } else {
        const T omb = T(1) - vs.beta;
        T fi[L::Q];
        T s0 = T(0), s1[3] = {T(0), T(0), T(0)};
        unroll<0, L::Q>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            fi[i] = load_pop<D, SOLIDS, PH, i>(f, mask, ev, ph, g, nb);
            if (!in_pminus<D, i>(nv)) {
                const T d = (fi[i] - T(1.5) * ftgt.template at<i>()) + T(0.5) * fst.template at<i>();
                s0 = s0 + d;
                unroll<0, D>([&](auto ia) {
                    constexpr int a = decltype(ia)::value;
                    if constexpr (L::c[i][a] == 1) s1[a] = s1[a] + d;
                    else if constexpr (L::c[i][a] == -1) s1[a] = s1[a] - d;
                });
            }
        });
        const T rloc = dv(own.e * own.r + omb * s0, own.e);
        T vloc[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int a = 0; a < D; ++a) vloc[a] = dv(own.r * own.w[a] + omb * s1[a], rloc);
        ProductForm<D, T> floc;
        eq_at<D>(own.e, rloc, vloc, ph.RT, floc);
        unroll<0, L::Q>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            const T neq = dv(ftgt.template at<i>() - floc.template at<i>(), omb);
            const T v = in_pminus<D, i>(nv)
                            ? neq + (T(1.5) * ftgt.template at<i>() - T(0.5) * fst.template at<i>())
                            : neq + fi[i];
            write_read_slot<D, SOLIDS, PH, i>(f, mask, ev, ph, g, nb, v);
        });
    }
}

}  // namespace lbm
