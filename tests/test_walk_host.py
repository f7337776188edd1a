"""The nonuniform-grid mover of the particle kernels (`walk` in
pic_common.hpp), compiled for the host: on random grids made of runs of
equal widths, every move must land where the physical displacement puts it
(fp64 reference: cell edges by cumulative sums), absorb exactly the moves
that leave the gap, keep offsets in [0, 1), and read the width tables only
inside [0, N).  The device intrinsics it uses (rounded add, subtract,
divide) are single IEEE operations and are stood in for by plain float
arithmetic."""
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

HARNESS = r'''
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>
static inline float __fsub_rn(float a, float b) { volatile float r = a - b; return r; }
static inline float __fadd_rn(float a, float b) { volatile float r = a + b; return r; }
static inline float __fdiv_rn(float a, float b) { volatile float r = a / b; return r; }
using std::fmaf;
template <class T> struct Checked {      // a table that aborts on an access outside [0, n)
    const T* p; int n;
    T operator[](int i) const { if (i < 0 || i >= n) { std::printf("out of bounds %d\n", i); std::exit(3); } return p[i]; }
};
@WALK@
int main() {
    std::mt19937_64 g(11);
    long bad = 0, moves = 0;
    for (int trial = 0; trial < 300; ++trial) {
        const int N = 2 + (int)(g() % 400);
        std::vector<double> w(N);
        for (int j = 0; j < N;) {
            const int len = 1 + (int)(g() % 50);
            const double wid = 0.2 + (double)(g() % 1000) / 250.0;
            for (int t = 0; t < len && j < N; ++t) w[j++] = wid;
        }
        double L = 0.0;
        for (double x : w) L += x;
        const double dx = L / N;
        std::vector<float> r(N);
        std::vector<uint32_t> run(N);
        std::vector<double> e(N + 1, 0.0);
        for (int k = 0; k < N; ++k) { r[k] = (float)(dx / w[k]); e[k + 1] = e[k] + w[k]; }
        for (int k = 0, a = 0; k < N; ++k)
            if (k + 1 == N || r[k + 1] != r[k]) {
                for (int t = a; t <= k; ++t) run[t] = (uint32_t)a | ((uint32_t)k << 16);
                a = k + 1;
            }
        const Checked<float> rc{r.data(), N};
        const Checked<uint32_t> uc{run.data(), N};
        std::uniform_real_distribution<double> U(0.0, 1.0);
        for (int q = 0; q < 2000; ++q) {
            int c = (int)(g() % N);
            float o = (float)U(g);
            if (o >= 1.0f) o = 0.0f;
            const float d = (float)((U(g) - 0.5) * 2.0 * ((g() % 4) == 0 ? N : 8.0));
            const double X = e[c] + (double)o * w[c] + (double)d * dx;
            walk(c, o, d, rc, uc, N);
            ++moves;
            const double tol = 1e-4 * dx * (1.0 + std::fabs((double)d));
            if (c < 0 || c >= N) {            // absorbed: must have left the gap
                if (X > tol && X < L - tol) ++bad;
                continue;
            }
            if (!(o >= 0.0f && o < 1.0f)) { ++bad; continue; }
            if (std::fabs(e[c] + (double)o * w[c] - X) > tol) ++bad;
        }
    }
    std::printf("%ld %ld\n", moves, bad);
    return bad != 0;
}
'''


def test_walk_matches_the_physical_move(tmp_path):
    src = open(os.path.join(ROOT, "paper_1310_5284_amd", "csrc", "pic_common.hpp")).read()
    m = re.search(r"template <class RP, class UP>\n__device__ __forceinline__ void walk\(.*?\n}\n",
                  src, re.S)
    assert m, "walk not found"
    fn = m.group(0).replace("__device__ __forceinline__", "static inline")
    prog = tmp_path / "walk.cpp"
    prog.write_text(HARNESS.replace("@WALK@", fn))
    exe = tmp_path / "walk"
    subprocess.check_call(["g++", "-O2", "-std=c++17", str(prog), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    moves, bad = map(int, out.stdout.split())
    assert moves == 600000 and bad == 0
