"""Planted-mistake check of the oracle's pins (CPU only; not collected by pytest).

Each mutant plants one plausible mistake in a copy of oracle/oracle.cpp (a
dropped term, a wrong factor, sign, index or operand, a swapped side), builds
it, and runs the oracle's CPU tests (tests/test_oracle_*.py) on the copy.  A
mutant is caught when any test fails.  The GPU library is not involved.

    python tests/mutation_check.py [--workers 6] [name,name,...]

About 30 minutes on 8 cores for the full list.
"""
import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (name, text in oracle.cpp, replacement); each text occurs exactly once
MUTANTS = [
 ("lame mu factor", "*mu = E / (2.0 * (1.0 + nu));", "*mu = E / (1.0 + nu);"),
 ("lame lambda denominator", "((1.0 + nu) * (1.0 - 2.0 * nu))", "((1.0 + nu) * (1.0 - nu))"),
 ("C shear = 2 mu", "for (int i = 3; i < 6; ++i) C[i][i] = mu;", "for (int i = 3; i < 6; ++i) C[i][i] = 2.0 * mu;"),
 ("grad N0 dropped term", "g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);\n  return det / 6.0;", "g[0][d] = -(g[1][d] + g[2][d]);\n  return det / 6.0;"),
 ("tet volume factor", "  return det / 6.0;\n}", "  return det / 2.0;\n}"),
 ("B row 4 index", "B[4][c + 1] = gz;", "B[4][c + 1] = gy;"),
 ("B row 5 operand", "B[5][c + 0] = gz;", "B[5][c + 0] = gx;"),
 ("inverse transposed", "for (int d = 0; d < 3; ++d) g[l][d] = inv[l - 1][d];", "for (int d = 0; d < 3; ++d) g[l][d] = inv[d][l - 1];"),
 ("smoothing weight V not Veff", "double w = c->el[j].Veff / S;\n        for (int r = 0; r < 6; ++r) eps[k][r] += w * eps_el[per * j + q][r];", "double w = c->el[j].V / S;\n        for (int r = 0; r < 6; ++r) eps[k][r] += w * eps_el[per * j + q][r];"),
 ("smoothing overwrite", "eps[k][r] += w * eps_el[per * j + q][r];", "eps[k][r] = w * eps_el[per * j + q][r];"),
 ("V_k missing 1/D", "      double Vk = S / c->D;\n      for (size_t i = 0; i < c->patch[k].size(); ++i) {", "      double Vk = S;\n      for (size_t i = 0; i < c->patch[k].size(); ++i) {"),
 ("force sign", "f[e.n[q / 3]][q % 3] += Vk * w * s;", "f[e.n[q / 3]][q % 3] -= Vk * w * s;"),
 ("force uses B^T eps", "for (int r = 0; r < 6; ++r) s += B[r][q] * sig[k][r];", "for (int r = 0; r < 6; ++r) s += B[r][q] * eps[k][r];"),
 ("mass from V", "c->m[e.n[l]] += c->rho * e.Veff / e.nn;", "c->m[e.n[l]] += c->rho * e.V / e.nn;"),
 ("mass split 1/3", "c->m[e.n[l]] += c->rho * e.Veff / e.nn;", "c->m[e.n[l]] += c->rho * e.Veff / 3.0;"),
 ("side fraction 1/8 <-> 7/8", "if (nodes_on_side == 1) return 0.125;", "if (nodes_on_side == 1) return 0.875;"),
 ("copy fraction side swapped", "c->el[t].Veff = side_fraction(4 - nb) * c->el[t].V;", "c->el[t].Veff = side_fraction(nb) * c->el[t].V;"),
 ("extra node starts at rest", "c->u.push_back(c->u[real]);", "c->u.push_back({0, 0, 0});"),
 ("crack area 2|2 factor", "return 0.25 * norm(cross(sub(x[A[1]], x[A[0]]), sub(x[Bn[1]], x[Bn[0]])));", "return 0.5 * norm(cross(sub(x[A[1]], x[A[0]]), sub(x[Bn[1]], x[Bn[0]])));"),
 ("crack area 1|3 factor", "return 0.125 * norm(cross(sub(x[q[1]], x[q[0]]), sub(x[q[2]], x[q[0]])));", "return 0.25 * norm(cross(sub(x[q[1]], x[q[0]]), sub(x[q[2]], x[q[0]])));"),
 ("delta_2 wrong nodes", "V3 d1 = stretch(N1, N2), d2 = stretch(N2, N3);", "V3 d1 = stretch(N1, N2), d2 = stretch(N1, N3);"),
 ("stretch test off", "if (d > 0.0) return du;", "if (d > -1e300) return du;"),
 ("G_I without 1/2", "*GI = 0.5 * (s3 * std::fabs(dot(d1, nI)) + s4 * std::fabs(dot(d2, nI)));", "*GI = (s3 * std::fabs(dot(d1, nI)) + s4 * std::fabs(dot(d2, nI)));"),
 ("sigma_G4 wrong edge", "double s4 = stress_term(sig[edge(N3, N4)].data(), nI, c->gsig);", "double s4 = stress_term(sig[edge(N1, N4)].data(), nI, c->gsig);"),
 ("n_I wrong vector", "V3 nI = unit(cross(sub(X3, X1), sub(X4, X2)));", "V3 nI = unit(cross(sub(X3, X1), sub(X4, X1)));"),
 ("principal projector not square-rooted", "return lmax * std::sqrt(p2);", "return lmax * p2;"),
 ("lone node wrong", "int lone = (b1 == b2) ? fl[0] : (b0 == b2) ? fl[1] : fl[2];", "int lone = (b1 == b2) ? fl[1] : (b0 == b2) ? fl[0] : fl[2];"),
 ("predictor a term", "u1[i][d] = c->u[i][d] + dt * c->v[i][d] + 0.5 * dt * dt * c->a[i][d];", "u1[i][d] = c->u[i][d] + dt * c->v[i][d] + dt * dt * c->a[i][d];"),
 ("velocity update explicit", "c->v[i][d] = c->v[i][d] + 0.5 * dt * (c->a[i][d] + an1);", "c->v[i][d] = c->v[i][d] + dt * an1;"),
 ("external work rule", "c->W += 0.5 * (rn + rn1) * c->F[i][d] * (u1[i][d] - c->u[i][d]);", "c->W += rn1 * c->F[i][d] * (u1[i][d] - c->u[i][d]);"),
 ("strain energy factor", "se += 0.5 * (Vsum[k] / c->D) * s;", "se += (Vsum[k] / c->D) * s;"),
 ("dissipation without Gc", "c->Ud += c->Gc * crack_area(x, e.mask);", "c->Ud += crack_area(x, e.mask);"),
 ("load ramp inverted", "if (c->ramp_t0 > 0.0 && t < c->ramp_t0) return t / c->ramp_t0;", "if (c->ramp_t0 > 0.0 && t < c->ramp_t0) return 1.0 - t / c->ramp_t0;"),
 ("bc displacement integral", "if (t0 > 0 && t <= t0) return t * t / (2.0 * t0);", "if (t0 > 0 && t <= t0) return t * t / t0;"),
 ("reaction sign of load", "R[b][d] = c->m[i] * c->a[i][d] + f[i][d] - r * c->F[i][d];", "R[b][d] = c->m[i] * c->a[i][d] + f[i][d] + r * c->F[i][d];"),
 ("hex smoothing 1/12 -> 1/6", "  c->D = 12.0;", "  c->D = 6.0;"),
 ("hex dN factor", "dN[i][1] = f[0] * sg[i][1] * f[2] / 8.0;", "dN[i][1] = f[0] * sg[i][1] * f[2] / 4.0;"),
 ("hex III G3 on the front face", "w3[j] = hex_mid(qa, j); w3[k] = -s;", "w3[j] = hex_mid(qa, j); w3[k] = s;"),
 ("hex IV pairs G3 with G2", "w3[i] = sg; w3[j] = hex_mid(qa, j);", "w3[i] = sg; w3[j] = hex_mid(qb, j);"),
 ("hex IV tilt toward the face", "      c[i] = sg;\n      c[k] = s;", "      c[i] = sg;\n      c[k] = -s;"),
 ("hex V G4 on the front face", "w4[i] = r; w4[k] = -s;", "w4[i] = r; w4[k] = s;"),
 ("hex VI corner on the far face", "    c[k] = s;\n    int w6[3]", "    c[k] = -s;\n    int w6[3]"),
 ("hex quad normal from sides", "nn = cross(sub(P4, P1), sub(P3, P2));", "nn = cross(sub(P2, P1), sub(P3, P1));"),
 ("hex G-II without 1/2", "if (k.pattern == 6) return 0.5 * s3 * (a1 + a2);", "if (k.pattern == 6) return s3 * (a1 + a2);"),
 ("hex G-I both stresses at G3", "return 0.5 * (s3 * a1 + s4 * a2);", "return 0.5 * (s3 * a1 + s3 * a2);"),
 ("hex stretch test off", "if (2.0 * dot(dX, du) + dot(du, du) > 0.0) return du;", "if (2.0 * dot(dX, du) + dot(du, du) > -1e300) return du;"),
 ("hex III keeps half", "return p < 3 ? 0.0 : 0.5;", "return p < 3 ? 0.5 : 0.5;"),
 ("hex prism keeps all", "return p < 3 ? 0.0 : 0.5;", "return p < 3 ? 0.0 : 1.0;"),
 ("hex ties to the later candidate", "if (G > best) { best = G; bmask = k.plane; bpat = k.pattern; }", "if (G >= best) { best = G; bmask = k.plane; bpat = k.pattern; }"),
 ("hex wedge index signs swapped", "return 3 + 4 * k + 2 * (c[a] > 0) + (c[b] > 0);", "return 3 + 4 * k + 2 * (c[b] > 0) + (c[a] > 0);"),
 ("hex face side swapped", "int axis = f / 2, side = (f & 1) ? 1 : -1, m = 0;", "int axis = f / 2, side = (f & 1) ? -1 : 1, m = 0;"),
 ("hex front into cracked hexes", "if (nb < 0 || c->smask[nb] >= 0) continue;\n      int qs[2]", "if (nb < 0) continue;\n      int qs[2]"),
 ("hex crack area from a side", "return 0.5 * norm(cross(sub(P[far], P[0]), sub(P[o[1]], P[o[0]])));", "return 0.5 * norm(cross(sub(P[far], P[0]), sub(P[o[1]], P[0])));"),
 ("hex crack area triangle factor", "if (n == 3) return 0.5 * norm(cross(sub(P[1], P[0]), sub(P[2], P[0])));", "if (n == 3) return norm(cross(sub(P[1], P[0]), sub(P[2], P[0])));"),
 ("uncut faces made fronts", "if (b0 == b1 && b1 == b2) continue;  // face not cut", "if (b0 == b1 && b1 == b2 && false) continue;"),
 ("front face index of the splitter", "r.face = c->nbr_face[s][f];", "r.face = f;"),
 ("erosion keeps half the volume", "par.Veff = 0.0;", "par.Veff = 0.5 * par.V;"),
 ("bc acceleration zero on the ramp", "? 1.0 / t0 : 0.0; }", "? 0.0 : 0.0; }"),
 ("critical step factor", "*dt_crit = 2.0 / std::sqrt(", "*dt_crit = 1.0 / std::sqrt("),
 ("replayed tet split twice", "      if (c->smask[e.tet] >= 0) continue;\n      e.pattern", "      e.pattern"),
 ("masses not rebuilt after splits", "  if (!evs.empty() && c->mode == 0 && c->D == 6.0) rebuild_masses(c);", "  (void)evs;"),
 ("adjoint: v sensitivity misses dt ub", "vb[i][d] = v1 + dt * u1;", "vb[i][d] = v1;"),
 ("adjoint: a sensitivity misses dt^2/2 ub", "ab[i][d] = 0.5 * dt * v1 + 0.5 * dt * dt * u1;", "ab[i][d] = 0.5 * dt * v1;"),
 ("adjoint: modulus term sign", "modulus_term(c, lam, us[s + 1], -1.0, Eb);", "modulus_term(c, lam, us[s + 1], 1.0, Eb);"),
 ("adjoint: modulus term at the final state", "modulus_term(c, lam, us[s + 1], -1.0, Eb);", "modulus_term(c, lam, us.back(), -1.0, Eb);"),
 ("adjoint: K term sign", "for (int d = 0; d < 3; ++d) ub[i][d] -= f[i][d];", "for (int d = 0; d < 3; ++d) ub[i][d] += f[i][d];"),
 ("adjoint: modulus weight dropped", "out[c->el[j].parent] += scale * Vk * (c->el[j].Veff / S) * q;", "out[c->el[j].parent] += scale * Vk * q;"),
 ("traction face area factor", "double A = 0.5 * norm(cross(sub(c->X[b], c->X[a]), sub(c->X[d], c->X[a])));", "double A = norm(cross(sub(c->X[b], c->X[a]), sub(c->X[d], c->X[a])));"),
 ("traction on one vertex only", "for (int k = 0; k < 3; ++k) c->F[n][k] += t[3 * f + k] * A / 3.0;", "for (int k = 0; k < 3; ++k) c->F[n][k] += q == 0 ? t[3 * f + k] * A : 0.0;"),
 ("traction components swapped", "for (int k = 0; k < 3; ++k) c->F[n][k] += t[3 * f + k] * A / 3.0;", "for (int k = 0; k < 3; ++k) c->F[n][k] += t[3 * f + (k + 1) % 3] * A / 3.0;"),
 ("bc velocity without its ramp", "double bc_vel(double t0, double t) { return (t0 > 0 && t <= t0) ? t / t0 : 1.0; }", "double bc_vel(double t0, double t) { return 1.0; }"),
 ("split neighbours taken as fronts", "if (nbt < 0 || c->smask[nbt] >= 0) continue;", "if (nbt < 0) continue;"),
 ("G_max is the last rather than the largest", "if (!any || best > c->Gmax) c->Gmax = best;", "c->Gmax = best;"),
 ("pattern I cuts off the wrong pair", "*maskI = (1 << lN2) | (1 << lN4);", "*maskI = (1 << lN2) | (1 << lN1);"),
 ("pattern II cuts off the wrong node", "*maskII = (1 << lN2);", "*maskII = (1 << lN4);"),
 ("initial acceleration ignores the ramp", "for (int d = 0; d < 3; ++d) c->a[i][d] = accel(c, i, r * c->F[i][d] - f[i][d]);", "for (int d = 0; d < 3; ++d) c->a[i][d] = accel(c, i, c->F[i][d] - f[i][d]);"),
 ("kinetic energy factor", "ke += 0.5 * c->m[i] * dot(c->v[i], c->v[i]);", "ke += c->m[i] * dot(c->v[i], c->v[i]);"),
 ("modulus smoothing weight by V", "    double w = c->el[j].Veff / S;\n    for (int r = 0; r < 6; ++r)\n      for (int q = 0; q < 6; ++q) Ck[r][q] += w * Cj[r][q];", "    double w = c->el[j].V / S;\n    for (int r = 0; r < 6; ++r)\n      for (int q = 0; q < 6; ++q) Ck[r][q] += w * Cj[r][q];"),
 ("copy takes a slot's modulus", "lame(c->Et[c->el[j].parent], c->nu, &lam, &mu);", "lame(c->Et[j < c->T0 ? j : 0], c->nu, &lam, &mu);"),
 ("reaction work without the trapezoid", "c->grp_W[g] += 0.5 * (c->bc_R[b][d] + R[b][d]) * (c->u[i][d] - u0[i][d]);", "c->grp_W[g] += R[b][d] * (c->u[i][d] - u0[i][d]);"),
 ("bc predictor one step late", "c->bc_uref[b][d] + c->bc_v0[b][d] * bc_disp(c->grp_t0[c->bc_group[b]], tn1);", "c->bc_uref[b][d] + c->bc_v0[b][d] * bc_disp(c->grp_t0[c->bc_group[b]], tn);"),
 ("no gap for equal principal stresses", "double gap = 1e-6 * amax;", "double gap = 0.0;"),
 ("hex Gauss points at the wrong abscissa", "const double a = 1.0 / std::sqrt(3.0);", "const double a = 0.5;"),
 ("1|3 crack area from the wrong side", "int big = (nb == 1) ? 0 : 1;", "int big = (nb == 1) ? 1 : 0;"),
 ("strain energy without 1/D", "se += 0.5 * (Vsum[k] / c->D) * s;", "se += 0.5 * Vsum[k] * s;"),
 ("masses not rebuilt after pre-splits", "  if (c->mode == 0) rebuild_masses(c);\n  c->need_init = true;", "  c->need_init = true;"),
 ("2|2 crack area from the wrong diagonals", "return 0.25 * norm(cross(sub(x[A[1]], x[A[0]]), sub(x[Bn[1]], x[Bn[0]])));", "return 0.25 * norm(cross(sub(x[A[1]], x[Bn[0]]), sub(x[Bn[1]], x[A[0]])));"),
 ("stretch test without its quadratic term", "double d = 2.0 * dot(dX, du) + dot(du, du);", "double d = 2.0 * dot(dX, du);"),
 ("pattern II wins ties", "if (GII > best) { best = GII; bmask = mII; bpat = 2; }", "if (GII >= best) { best = GII; bmask = mII; bpat = 2; }"),
 ("later face wins ties", "if (GI > best) { best = GI; bmask = mI; bpat = 1; }", "if (GI >= best) { best = GI; bmask = mI; bpat = 1; }"),
 ("fronts visited in reverse face order", "return x.c != y.c ? x.c < y.c : x.face < y.face;\n  });\n  return fr;\n}\n\n// Release rates", "return x.c != y.c ? x.c < y.c : x.face > y.face;\n  });\n  return fr;\n}\n\n// Release rates"),
 ("hex fronts in reverse face order", "return x.c != y.c ? x.c < y.c : x.face < y.face;\n  });\n  return fr;\n}\n\n// Area of the crack", "return x.c != y.c ? x.c < y.c : x.face > y.face;\n  });\n  return fr;\n}\n\n// Area of the crack"),
 ("Griffith test strict", "if (best >= c->Gc) out.push_back", "if (best > c->Gc) out.push_back"),
 ("tie gap too narrow", "double gap = 1e-6 * amax;", "double gap = 1e-10 * amax;"),
 ("tie gap too wide", "double gap = 1e-6 * amax;", "double gap = 1e-5 * amax;"),
 ("hex inverse Jacobian entry transposed", "double inv[3][3];  // J^{-1}\n  inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;\n  inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;", "double inv[3][3];  // J^{-1}\n  inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;\n  inv[0][1] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;"),
 ("hex edge point at the element centre", "for (int d = 0; d < 3; ++d) xi[d] = 0.5 * (sg[p0][d] + sg[p1][d]);", "for (int d = 0; d < 3; ++d) xi[d] = 0.0 * (sg[p0][d] + sg[p1][d]);"),
 ("hex patch entries on the wrong edge point", "int q = per == 1 ? 0 : c->patch_q[k][i];", "int q = per == 1 ? 0 : (c->patch_q[k][i] + 1) % 12;"),
]


def make_copy(dst):
    skip = shutil.ignore_patterns("*.so", "__pycache__", "csrc")
    for d in ("oracle", "tests", "paper_2508_04076_amd"):
        shutil.copytree(os.path.join(ROOT, d), os.path.join(dst, d), ignore=skip)


def run_one(mutant, work, src, tests):
    name, a, b = mutant
    if src.count(a) != 1:
        return name, f"NOT APPLIED (text found {src.count(a)} times)"
    open(os.path.join(work, "oracle", "oracle.cpp"), "w").write(src.replace(a, b))
    lib = os.path.join(work, "oracle", "liboracle.so")
    if os.path.exists(lib):
        os.remove(lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *tests],
                       cwd=work, capture_output=True, text=True, timeout=900)
    if r.returncode == 0:
        return name, "SURVIVED"
    failed = [l for l in r.stdout.splitlines() if l.startswith("FAILED")]
    which = failed[0].split("::")[-1].split(" ")[0] if failed else f"exit {r.returncode}"
    return name, f"caught by {which}"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="?", help="comma-separated mutant names (default: all)")
    ap.add_argument("--workers", type=int, default=6)
    args = ap.parse_args()
    muts = MUTANTS
    if args.names:
        want = args.names.split(",")
        muts = [m for m in MUTANTS if m[0] in want]
    src = open(os.path.join(ROOT, "oracle", "oracle.cpp")).read()
    tests = sorted(os.path.join("tests", f) for f in os.listdir(os.path.join(ROOT, "tests"))
                   if f.startswith("test_oracle") and f.endswith(".py"))
    W = max(1, min(args.workers, len(muts)))
    out = {}
    with tempfile.TemporaryDirectory(prefix="oracle_mutants_") as tmp:
        works = []
        for w in range(W):
            d = os.path.join(tmp, f"w{w}")
            make_copy(d)
            works.append(d)

        def worker(w):
            return [run_one(m, works[w], src, tests) for m in muts[w::W]]

        with cf.ThreadPoolExecutor(W) as ex:
            for res in ex.map(worker, range(W)):
                out.update(res)
    for name, _, _ in muts:
        print(f"{name:42s} {out[name]}", flush=True)
    caught = sum(v.startswith("caught") for v in out.values())
    print(f"caught {caught} of {len(muts)}")
    return 0 if caught == len(muts) else 1


if __name__ == "__main__":
    sys.exit(main())
