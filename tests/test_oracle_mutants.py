"""Planted mistakes in the oracle: each case copies the oracle package (oracle.c and its
Python side), makes one plausible mistake in the copy (a dropped term, a flipped sign, a
wrong index or constant, swapped operands), builds it with the oracle's own gcc flags and
runs the pin tests of the part it touches against it, the copy imported in place of the
oracle.  A mistake that every pin let through would be one the pins cannot see, so each
case requires at least one pin to fail, and an unchanged copy run the same way must pass
them all.  Tests that compare the GPU library with the oracle are left out (the library is
not what is pinned here).  CPU only."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(HERE)
ORACLE = os.path.join(REPO, "oracle")

CLOUD = "test_oracle_cloud.py"
DESC = "test_oracle_descriptor.py"
NET = "test_oracle_network.py"
TRACE = "test_oracle_tracer.py"
PHASE = "test_oracle_phase.py"
LIGHTS = "test_oracle_lights.py"
RECORDS = "test_oracle_records.py"
FP8 = "test_oracle_fp8.py"
MLP = "test_oracle_mlp.py"

# (name, pin files, text (occurs once in the file), replacement, the passage it breaks)
MUTANTS = [
    ("mean_over_all_voxels", [CLOUD],
     "*mean_mu_t = sum / (double)cnt;", "*mean_mu_t = sum / (double)n;",
     "Sec. 4.2: the mean extinction is taken over the non-empty voxels"),
    ("mip_sample_not_voxel_centred", [CLOUD],
     "double t = ((double)j + 0.5) - ((double)m + 0.5) * s;",
     "double t = (double)j - (double)m * s;",
     "Sec. 6: level samples sit at the centres of the coarser voxels"),
    ("mip_truncated_at_two_sigma", [CLOUD],
     "    if (fabs(t) > 3.0 * s)\n        return 0.0;",
     "    if (fabs(t) > 2.0 * s)\n        return 0.0;",
     "Sec. 6: the Gaussian is cut at three standard deviations"),
    ("mip_norm_level0_short", [CLOUD],
     "for (int t = -3; t <= 3; ++t)", "for (int t = -2; t <= 2; ++t)",
     "Sec. 6: the normaliser sums the kernel over every offset within three sigma"),
    ("mip_norm_integer_offsets", [CLOUD],
     "double t = (double)k + 0.5;", "double t = (double)k;",
     "Sec. 6: above level 0 the base voxel centres sit at half-integer offsets"),
    ("frame_x_reversed", [DESC],
     "cross3(w, Z, xp);", "cross3(Z, w, xp);",
     "Sec. 4.2: the x axis of the local frame is w x l, normalised"),
    ("gamma_of_the_reversed_view", [DESC],
     "double c = dot3(w, Z);", "double c = -dot3(w, Z);",
     "Sec. 4.2: gamma is the angle between view and light direction"),
    ("stencil_z_span_halved", [DESC],
     "o[2] = -1.0 + 0.5 * iz;", "o[2] = -1.0 + 0.25 * iz;",
     "Sec. 4.2, Fig. 5: the stencil reaches three mean free paths towards the light"),
    ("level_scale_off_by_one", [DESC],
     "double s = ldexp(1.0, k) / mean_mu_t;", "double s = ldexp(1.0, k + 1) / mean_mu_t;",
     "Sec. 4.2: level k is scaled by 2^(k-1) mean free paths"),
    ("trilinear_y_weights_swapped", [DESC],
     "(dy ? f[1] : 1.0 - f[1]) *\n                           (dz ? f[2] : 1.0 - f[2]);\n"
     "                acc += w * lv[",
     "(dy ? 1.0 - f[1] : f[1]) *\n                           (dz ? f[2] : 1.0 - f[2]);\n"
     "                acc += w * lv[",
     "Sec. 4.2: densities are read by trilinear interpolation"),
    ("trilinear_x_z_transposed", [DESC],
     "acc += w * lv[(c[2] * my + c[1]) * mx + c[0]];",
     "acc += w * lv[(c[0] * my + c[1]) * mx + c[2]];",
     "Sec. 4.2: the level grid is indexed x fastest"),
    ("sample_not_voxel_centred", [DESC],
     "u[a] = (q - aabb_min[a]) / hm - 0.5;", "u[a] = (q - aabb_min[a]) / hm;",
     "Sec. 6: voxel-centred interpolation in each mip level"),
    ("fallback_box_too_short", [DESC],
     "(c & 4) ? 3.0 : -1.0", "(c & 4) ? 1.0 : -1.0",
     "Sec. 4.2: the level-1 stencil box reaches three mean free paths towards the light"),
    ("residual_dropped", [NET],
     "a[r] = acc + op[r];", "a[r] = acc;",
     "Sec. 4.3, Fig. 6: each block adds its input to the second layer"),
    ("gamma_not_fed_to_blocks", [NET],
     "            for (int c = 0; c < 226; ++c)\n                acc += vr[c] * zk[c];",
     "            for (int c = 0; c < 225; ++c)\n                acc += vr[c] * zk[c];",
     "Sec. 4.3: every block reads its stencil level and gamma"),
    ("output_relu_dropped", [NET],
     "ho[r] = relu(acc);", "ho[r] = acc;",
     "Sec. 4.3: the trailing layers, the output one included, are ReLUs"),
    ("loss_not_averaged", [NET],
     "*loss = L / (double)B;", "*loss = L;",
     "Sec. 5.2: the loss is the mean over the batch"),
    ("loss_chain_rule_through_log_dropped", [NET],
     "double dg = 2.0 * r / ((double)B * (1.0 + gv));", "double dg = 2.0 * r / (double)B;",
     "Sec. 5.2: the loss compares log(1 + g) with log(1 + L)"),
    ("residual_gradient_dropped", [NET],
     "                dnext[c] = da[c];", "                dnext[c] = 0.0;",
     "Sec. 4.3: the residual path carries the gradient to the previous block"),
    ("adam_without_bias_correction", [NET],
     "double mh = m[i] / c1;", "double mh = m[i];",
     "Sec. 5.2 (Adam, Kingma and Ba): bias-corrected first moment"),
    ("philox_second_key_constant", [NET],
     "k1 += 0xBB67AE85u;", "k1 += 0x9E3779B9u;",
     "Philox4x32-10 (Salmon et al.): the second Weyl key increment"),
    ("tracer_density_x_z_transposed", [TRACE],
     "density_at(M->d, M->dtype, (c[2] * M->ny + c[1]) * M->nx + c[0])",
     "density_at(M->d, M->dtype, (c[0] * M->ny + c[1]) * M->nx + c[2])",
     "Sec. 3: the tracer reads the same x-fastest density grid"),
    ("tracer_density_z_weights_swapped", [TRACE],
     "(dz ? f[2] : 1.0 - f[2]);\n                acc += w * density_at(",
     "(dz ? 1.0 - f[2] : f[2]);\n                acc += w * density_at(",
     "Sec. 3: the tracer interpolates the density trilinearly"),
    ("tracer_density_x_weights_swapped", [TRACE],
     "double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) *\n"
     "                           (dz ? f[2] : 1.0 - f[2]);\n                acc += w * density_at(",
     "double w = (dx ? 1.0 - f[0] : f[0]) * (dy ? f[1] : 1.0 - f[1]) *\n"
     "                           (dz ? f[2] : 1.0 - f[2]);\n                acc += w * density_at(",
     "Sec. 3: the tracer interpolates the density trilinearly"),
    ("hg_sign_of_g", [TRACE],
     "double den = 1.0 + g * g - 2.0 * g * mu;", "double den = 1.0 + g * g + 2.0 * g * mu;",
     "Henyey-Greenstein: forward scattering for g > 0"),
    ("hg_sample_backwards", [TRACE],
     "double c = (1.0 + g * g - s * s) / (2.0 * g);",
     "double c = (s * s - 1.0 - g * g) / (2.0 * g);",
     "Henyey-Greenstein inverse CDF: the sampled cosine has mean g"),
    ("delta_tracking_accepts_null", [TRACE],
     "if (rng_u(r) * M->maj < mu_at(M, p)) {", "if (rng_u(r) * M->maj > mu_at(M, p)) {",
     "Sec. 3: delta tracking takes a real collision with probability mu / majorant"),
    ("ratio_tracking_weight_inverted", [TRACE],
     "T *= 1.0 - mu_at(M, p) / M->maj;", "T *= mu_at(M, p) / M->maj;",
     "ratio tracking multiplies by the null-collision probability"),
    ("albedo_roulette_inverted", [TRACE],
     "if (rng_u(r) >= tp->albedo)\n            break;", "if (rng_u(r) < tp->albedo)\n            break;",
     "Sec. 3: a path survives a collision with probability equal to the albedo"),
    ("sun_cosine_sign", [TRACE],
     "double mu = -dot3(wh, wl);", "double mu = dot3(wh, wl);",
     "Sec. 3: next-event estimation towards the sun, cosine of the scattering angle"),
    ("chop_albedo_not_renormalised", [PHASE],
     "*albedo = a * (1.0 - g_removed) / s;", "*albedo = a * (1.0 - g_removed);",
     "Sec. 3.1: the thinner medium keeps the scattering left after the chop"),
    ("phase_table_not_interpolated", [PHASE],
     "return t->p[i] + f * (t->p[i + 1] - t->p[i]);", "return t->p[i];",
     "Sec. 3.1: the tabulated phase function is linear in theta between nodes"),
    ("phase_table_sample_linear_in_u", [PHASE],
     "t = (-fa + sqrt(fa * fa + (fb - fa) * q * (fa + fb))) / (fb - fa);", "t = q;",
     "Sec. 3.1: theta inside a node interval follows the linear density p sin(theta)"),
    ("first_collision_weight_not_rescaled", [PHASE],
     "return (1.0 - g_removed_first) / (1.0 - g_removed);", "return 1.0 - g_removed_first;",
     "Sec. 3.1: the full function at the first collision, in the thinner medium"),
    ("camera_direct_cosine_sign", [TRACE, PHASE, LIGHTS],
     "direct = ph_eval(tp->g, 1, -dot3(w, wl)) * ratio_track(M, x, wl, r) * tp->irradiance;",
     "direct = ph_eval(tp->g, 1, dot3(w, wl)) * ratio_track(M, x, wl, r) * tp->irradiance;",
     "Sec. 4.4: single scattering at a camera ray's first collision"),
    ("adaptive_variance_of_a_sample", [RECORDS],
     "vm = fmax(0.0, (s2 - n * mean * mean) / (n - 1)) / n;",
     "vm = fmax(0.0, (s2 - n * mean * mean) / (n - 1));",
     "Sec. 5.1: records are traced until the mean's own error is small"),
    ("adaptive_rule_on_the_variance", [RECORDS],
     "if (zq * sqrt(vm) <= rel * fabs(mean))", "if (zq * vm <= rel * fabs(mean))",
     "Sec. 5.1: the stopping rule compares a standard error with the mean"),
    ("light_weight_dropped", [LIGHTS],
     "sum += tp->set->w[j] * ph_eval(tp->g, 0, mu) * T * tp->irradiance;",
     "sum += ph_eval(tp->g, 0, mu) * T * tp->irradiance;",
     "a light set picks light j with probability proportional to its weight"),
]


PY_MUTANTS = [
    ("e4m3_ties_round_up", [FP8],
     "np.where(hi % 2 == 0, hi, lo)", "hi",
     "OCP E4M3: ties go to the even code"),
    ("e4m3_subnormal_scale", [FP8],
     "return m * 2.0 ** -9 if e == 0", "return m * 2.0 ** -10 if e == 0",
     "OCP E4M3: subnormals are m 2^-9"),
    ("mlp_relu_gate_dropped", [MLP],
     "d = d * (pres[l] > 0)", "d = d",
     "Sec. 7: every layer of the comparison networks is a ReLU"),
    ("mlp_loss_chain_rule_dropped", [MLP],
     "d = (2.0 * r / (B * (1.0 + g)))[:, None]", "d = (2.0 * r / B)[:, None]",
     "Sec. 5.2: the loss compares log(1 + g) with log(1 + L)"),
    ("phase_cdf_left_sums", [PHASE],
     "np.cumsum(0.5 * (f[1:] + f[:-1]) * (np.pi / (n - 1)))",
     "np.cumsum(f[:-1] * (np.pi / (n - 1)))",
     "Sec. 5.1: the table's cdf is the trapezoid rule on 2 pi p sin(theta)"),
    ("phase_chop_zeroes_the_peak", [PHASE],
     "q[:ic] = q[ic]", "q[:ic] = 0.0",
     "Sec. 5.1: the chopped function is held constant below the chop angle"),
    ("light_threshold_truncated", [LIGHTS],
     "t = int(np.floor(run / total * 16777216.0 + 0.5))",
     "t = int(np.floor(run / total * 16777216.0))",
     "light selection: thresholds are the running sums rounded to nearest"),
    ("light_weight_of_the_running_sum", [LIGHTS],
     "w[j] = E[j] / ((t - prev) / 16777216.0)", "w[j] = E[j] / (t / 16777216.0)",
     "light selection: the weight divides by the light's own probability"),
]

CASES = [("oracle.c",) + m for m in MUTANTS] + [("__init__.py",) + m for m in PY_MUTANTS]
GCC = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE",
       "-ffp-contract=off"]


def make_copy(d, fname=None, old=None, new=None):
    """Copies the oracle package into d/oracle with `old` replaced by `new` in `fname`
    (no change when fname is None) and builds its library."""
    pkg = os.path.join(d, "oracle")
    os.makedirs(pkg)
    for f in ("oracle.c", "__init__.py"):
        with open(os.path.join(ORACLE, f)) as fh:
            text = fh.read()
        if f == fname:
            assert text.count(old) == 1, f"the mutated text must occur once in {f}"
            text = text.replace(old, new)
        with open(os.path.join(pkg, f), "w") as fh:
            fh.write(text)
    subprocess.run(GCC + [os.path.join(pkg, "oracle.c"), "-o", os.path.join(pkg, "liboracle.so"),
                          "-lm"], check=True)


def run_pins(d, files):
    """Runs the pin files with d/oracle imported as the oracle; returns pytest's exit code
    and its output."""
    args = ["-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu", "-k", "not library"]
    args += [os.path.join(HERE, f) for f in files]
    code = ("import sys; sys.path.insert(0, %r); import oracle; "
            "assert oracle.__file__.startswith(%r), oracle.__file__; "
            "import pytest; sys.exit(pytest.main(%r))" % (d, d, args))
    r = subprocess.run([sys.executable, "-c", code], cwd=REPO, capture_output=True, text=True,
                       timeout=900, env=dict(os.environ, OMP_NUM_THREADS="2"))
    return r.returncode, r.stdout + r.stderr


ALL_PINS = sorted({f for c in CASES for f in c[2]})


@pytest.fixture(scope="module")
def outcomes(tmp_path_factory):
    """(exit code, output) of every case and of the unchanged copy, run side by side (each
    case is its own process)."""
    base = tmp_path_factory.mktemp("mutants")

    def one(i):
        d = str(base / f"c{i}")
        os.makedirs(d)
        if i < 0:
            make_copy(d)
            return run_pins(d, ALL_PINS)
        fname, _, files, old, new, _ = CASES[i]
        make_copy(d, fname, old, new)
        return run_pins(d, files)

    idx = [-1] + list(range(len(CASES)))
    with ThreadPoolExecutor(max_workers=max(1, min(6, (os.cpu_count() or 2) - 1))) as ex:
        return dict(zip(idx, ex.map(one, idx)))


def test_unchanged_copy_passes_every_pin(outcomes):
    rc, out = outcomes[-1]
    assert rc == 0, out[-3000:]


@pytest.mark.parametrize("i", range(len(CASES)), ids=[c[1] for c in CASES])
def test_pins_catch_the_planted_mistake(outcomes, i):
    _, name, _, _, _, passage = CASES[i]
    rc, out = outcomes[i]
    # exit code 1: tests ran and at least one failed (2 and above are usage or collection
    # errors, which would not show that a pin saw the mistake)
    assert rc == 1, f"{name} ({passage}) passed every pin:\n{out[-2000:]}"
    assert " failed" in out
