"""The oracle's pins must catch plausible mistakes in it.

Each case plants one mistake in a copy of the oracle source (a dropped term, a wrong sign,
index, rule or constant), builds it with gcc on the CPU, and runs the pin that should catch
it against the broken build; that pin must fail.  The exact boundary convention of the
minimum image (v >= L/2 versus v > L/2) is not listed: it is unobservable (the absolute
value used by the walk is the same, and the pair force is zero at r = L/2 >= r_cut).
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "treepm_oracle.c")

PAIR = "tests/test_oracle_pair.py"
TREE = "tests/test_oracle_tree.py"

MUTANTS = [
    ("g1_coefficient", "48.0 * R7 - 21.0 * R8) / 140.0", "48.0 * R7 - 20.0 * R8) / 140.0",
     PAIR + "::test_g_is_s2_cloud_complement"),
    ("g2_coefficient", "- 840.0 * R4", "- 841.0 * R4", PAIR + "::test_g_branch2_factored"),
    ("g_branch_point", "if (R < 1.0)\n", "if (R <= 0.9)\n", PAIR + "::test_g_is_s2_cloud_complement"),
    ("wrap_dropped", "if (v < -h) return v + L;", "if (v < -h) return v;",
     PAIR + "::test_two_body_across_boundary"),
    ("softening_dropped", "double s2 = r2 + eps2;", "double s2 = r2;",
     PAIR + "::test_two_body_across_boundary"),
    ("force_sign", "acc[0] += f * d[0];", "acc[0] -= f * d[0];",
     PAIR + "::test_two_body_across_boundary"),
    ("eta_is_rcut", "double eta = 0.5 * r_cut, eps2 = eps * eps;\n#ifdef _OPENMP\n    if (nthreads > 0) omp_set_num_threads(nthreads);\n#pragma omp parallel for schedule(dynamic, 64)\n#endif\n    for (int64_t i = 0; i < n; ++i) {\n        double acc[3] = {0.0, 0.0, 0.0};\n        for (int64_t j = 0; j < n; ++j) {",
     "double eta = r_cut, eps2 = eps * eps;\n#ifdef _OPENMP\n    if (nthreads > 0) omp_set_num_threads(nthreads);\n#pragma omp parallel for schedule(dynamic, 64)\n#endif\n    for (int64_t i = 0; i < n; ++i) {\n        double acc[3] = {0.0, 0.0, 0.0};\n        for (int64_t j = 0; j < n; ++j) {",
     PAIR + "::test_zero_at_and_beyond_cutoff"),
    ("key_axis_order", "k |= ((q[0] >> b) & 1u) << (3 * b + 2);", "k |= ((q[0] >> b) & 1u) << (3 * b);",
     TREE + "::test_keys_hand_computed"),
    ("sort_unstable", "return (p->idx < q->idx) ? -1 : (p->idx > q->idx) ? 1 : 0;",
     "return (p->idx < q->idx) ? 1 : (p->idx > q->idx) ? -1 : 0;",
     TREE + "::test_sort_is_stable_key_sort"),
    ("leaf_rule", "if (nd.count < t->n_leaf || nd.level >= ORC_MAXLEVEL)",
     "if (nd.count <= t->n_leaf || nd.level >= ORC_MAXLEVEL)", TREE + "::test_tree_invariants"),
    ("com_not_divided", "nd->com[a] = S[a] / M;", "nd->com[a] = S[a];",
     TREE + "::test_tree_invariants"),
    ("group_rule", "if (nd->nchild == 0 || nd->count <= t->n_crit) return push_group(t, u);",
     "if (nd->nchild == 0 || nd->count < t->n_crit) return push_group(t, u);",
     TREE + "::test_groups_rule"),
    ("group_centre", "g->xg[a] = ((double)ic[a] + 0.5) * l;", "g->xg[a] = ((double)ic[a]) * l;",
     TREE + "::test_groups_rule"),
    ("bbox_half_size", "g->hg[a] = (hi[a] - lo[a]) * 0.5;", "g->hg[a] = (hi[a] - lo[a]) * 0.4;",
     TREE + "::test_lists_equal_brute_force_frontier"),
    ("prune_uses_full_side", "- (half + g->hg[a]);", "- (l + g->hg[a]);",
     TREE + "::test_lists_equal_brute_force_frontier"),
    ("accept_not_squared", "if (l * l < th2 * D && G > 0.0)", "if (l < th2 * D && G > 0.0)",
     TREE + "::test_lists_equal_brute_force_frontier"),
    ("accept_guard_dropped", "if (l * l < th2 * D && G > 0.0)", "if (l * l < th2 * D)",
     TREE + "::test_lists_never_accept_a_node_holding_the_group"),
    ("accept_on_tie", "if (l * l < th2 * D && G > 0.0)", "if (l * l <= th2 * D && G > 0.0)",
     TREE + "::test_opening_tie_opens_the_node"),
    ("leaf_particles_skipped", "for (int64_t k = nd->first; k < nd->first + nd->count; ++k)\n            if (elist_push(out, k, 0)) return -1;",
     "for (int64_t k = nd->first + 1; k < nd->first + nd->count; ++k)\n            if (elist_push(out, k, 0)) return -1;",
     TREE + "::test_theta_zero_is_direct_sum"),
    ("theta_r_inverted", "double th = theta0 / sqrt(s);", "double th = theta0 * sqrt(s);",
     TREE + "::test_theta_r_closed_forms"),
    ("theta_r_without_g_cost", "double s = R * orc_g_p3m(R);", "double s = R;",
     TREE + "::test_distance_opening_beats_fixed_in_uniform_limit"),
    ("theta_r_zero_where_rg_vanishes", "if (!(s > 0.0)) return theta_max;",
     "if (!(s > 0.0)) return 0.0;", TREE + "::test_theta_r_cap"),
    ("theta_r_no_sqrt", "double th = theta0 / sqrt(s);", "double th = theta0 / s;",
     TREE + "::test_theta_r_closed_forms"),
    ("theta_r_eta_is_rcut", "double R = r / eta;", "double R = r / (2.0 * eta);",
     TREE + "::test_theta_r_closed_forms"),
    ("theta_r_without_g", "double s = R * orc_g_p3m(R);", "double s = R;",
     TREE + "::test_theta_r_closed_forms"),
    ("theta_r_uncapped", "return th < theta_max ? th : theta_max;", "return th;",
     TREE + "::test_theta_r_cap"),
    ("opening_distance_squared", "orc_theta_r(sqrt(D), 0.5 * t->r_cut,",
     "orc_theta_r(D, 0.5 * t->r_cut,",
     TREE + "::test_distance_opening_lists_equal_brute_force_frontier"),
    ("quad_trace_half_dropped", "0.5 * trQ * d[a] * u", "trQ * d[a] * u",
     TREE + "::test_quadrupole_cell_is_third_order"),
    ("quad_w_sign", "- 6.0 * g1 * p / (eta * r)", "+ 6.0 * g1 * p / (eta * r)",
     TREE + "::test_quadrupole_cell_is_third_order"),
    ("quad_g2_coefficient", "2016.0 * R5 - 1176.0 * R6", "2016.0 * R5 - 1170.0 * R6",
     TREE + "::test_cutoff_derivatives"),
    ("quad_g1_branch2", "336.0 * R6 + 56.0 * R7) / 140.0;", "336.0 * R6 + 57.0 * R7) / 140.0;",
     TREE + "::test_cutoff_derivatives"),
    ("quad_eta_power", "g2 * q / (eta * eta * r2)", "g2 * q / (eta * r2)",
     TREE + "::test_quadrupole_cell_is_third_order"),
    ("quad_moment_offdiag", "Q[3] += m * dx * dy;", "Q[3] += m * dx * dz;",
     TREE + "::test_node_second_moments"),
    ("quad_not_applied", "if (t->quadrupole && isc[q]) pair_quad(",
     "if (0 && isc[q]) pair_quad(", TREE + "::test_quadrupole_tree_force_is_more_accurate"),
    ("sample_interactions_without_count", "inter += l.n * t->groups[gi].count;",
     "inter += l.n;", TREE + "::test_walk_force_sample_equals_full_walk_and_force"),
    ("sample_theta_not_squared",
     "double rc2 = t->r_cut * t->r_cut, th2 = t->theta * t->theta;\n    double eta = 0.5 * t->r_cut, eps2 = t->eps * t->eps;\n    int64_t inter = 0, parts = 0;",
     "double rc2 = t->r_cut * t->r_cut, th2 = t->theta;\n    double eta = 0.5 * t->r_cut, eps2 = t->eps * t->eps;\n    int64_t inter = 0, parts = 0;",
     TREE + "::test_walk_force_sample_equals_full_walk_and_force"),
    ("sample_scale_without_g", "                        pair_mag(d, mj, eta, eps2, &s, &sn);\n                    }\n                    mag[t->idx[k]] = s;\n                    newt[t->idx[k]] = sn;\n                }\n            }",
     "                        pair_mag(d, mj, eta, eps2, &sn, &s);\n                    }\n                    mag[t->idx[k]] = s;\n                    newt[t->idx[k]] = sn;\n                }\n            }",
     TREE + "::test_walk_force_sample_equals_full_walk_and_force"),
    ("set_theta_keeps_lists", "    t->theta = theta;\n    free(t->list_off);", "    t->theta = theta;\n    return 0;\n    free(t->list_off);",
     TREE + "::test_walk_force_sample_equals_full_walk_and_force"),
    ("opening_angle_not_squared", "        th2 = th * th;\n", "        th2 = th;\n",
     TREE + "::test_distance_opening_lists_equal_brute_force_frontier"),
]


PM = "tests/test_oracle_pm.py"
PY_MUTANTS = [  # (name, file under oracle/, old, new, pin)
    ("pm_fd_second_order", "pm.py", "(2.0 / 3.0) * (p1 - m1) - (1.0 / 12.0) * (p2 - m2)",
     "0.5 * (p1 - m1)", PM + "::test_converges_to_exact_long_range_force"),
    ("pm_window_once", "pm.py", "/ (W[pos] ** 2)", "/ W[pos]",
     PM + "::test_accuracy_at_the_papers_split"),
    ("pm_tsc_centre_weight", "pm.py", "0.75 - d * d", "0.7 - d * d",
     PM + "::test_tsc_cloud_closed_forms"),
    ("pm_nearest_point", "pm.py", "i0 = np.floor(u + 0.5)", "i0 = np.floor(u)",
     PM + "::test_tsc_cloud_closed_forms"),
    ("pm_interp_mirrored", "pm.py", "wt = w[:, 0, a] * w[:, 1, b] * w[:, 2, c]",
     "wt = w[:, 0, 2 - a] * w[:, 1, b] * w[:, 2, c]", PM + "::test_momentum_is_conserved"),
    ("pm_potential_units", "pm.py", "* (n ** 3) / L ** 3", "* (n ** 3) / L ** 2",
     PM + "::test_scaling_with_box_size"),
    ("pm_green_sign", "pm.py", "G[pos] = kern.phi_hat(uniq)[inv] / (W[pos] ** 2)",
     "G[pos] = -kern.phi_hat(uniq)[inv] / (W[pos] ** 2)", PM + "::test_short_plus_pm_is_ewald"),
    ("pm_mesh_spacing", "pm.py", "    h = L / phi.shape[0]\n", "    h = 2.0 * L / phi.shape[0]\n",
     PM + "::test_converges_to_exact_long_range_force"),
]


@pytest.mark.parametrize("name,fname,old,new,pin", PY_MUTANTS, ids=[m[0] for m in PY_MUTANTS])
def test_pin_catches_planted_mistake_py(tmp_path, name, fname, old, new, pin):
    """The same for the Python parts of the oracle: a mutated copy of the package is put
    first on the import path of the pin's process."""
    pkg = tmp_path / "oracle"
    shutil.copytree(os.path.join(ROOT, "oracle"), pkg,
                    ignore=shutil.ignore_patterns("__pycache__"))
    src = (pkg / fname).read_text()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    (pkg / fname).write_text(src.replace(old, new, 1))
    env = dict(os.environ, TREEPM_ORACLE_PKG=str(tmp_path))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, pin)], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 1, f"{name} survived {pin}:\n{r.stdout[-2000:]}"


@pytest.mark.parametrize("name,old,new,pin", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pin_catches_planted_mistake(tmp_path, name, old, new, pin):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mutated = src.replace(old, new, 1)
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(mutated)
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
                    "-ffp-contract=off", str(c), "-o", str(so), "-lm"], check=True)
    env = dict(os.environ, TREEPM_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, pin)], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 1, f"{name} survived {pin}:\n{r.stdout[-2000:]}"
