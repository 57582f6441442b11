"""The serving pool allocator (host-side first-fit over one device block),
compiled on the CPU with g++ and exercised by a randomised harness: blocks
never overlap, accounting is exact, freed neighbours coalesce, and a fully
freed pool is one block again."""
import os
import subprocess

HARNESS = r'''
#include "mc_pool.hpp"
#include <cstdio>
#include <random>
#include <vector>
#include <algorithm>
using mc::Pool;
int main() {
    std::mt19937_64 rng(7);
    for (int trial = 0; trial < 50; ++trial) {
        const int64_t size = (int64_t)(1 + rng() % 4096) * 256 + (int64_t)(rng() % 255);
        Pool p(size);
        if (p.size() % 256 != 0 || p.size() > size) { std::puts("FAIL size"); return 1; }
        std::vector<std::pair<int64_t,int64_t>> live;
        int64_t used = 0;
        for (int op = 0; op < 2000; ++op) {
            if (live.empty() || rng() % 3 != 0) {
                const int64_t want = 1 + (int64_t)(rng() % (size / 8 + 1));
                const int64_t off = p.alloc(want);
                if (off < 0) {
                    if (p.largest_free() >= Pool::round_up(want)) { std::puts("FAIL refused"); return 1; }
                    continue;
                }
                const int64_t len = Pool::round_up(want);
                if (off % 256 || off + len > p.size()) { std::puts("FAIL bounds"); return 1; }
                for (auto &b : live)
                    if (off < b.first + b.second && b.first < off + len) { std::puts("FAIL overlap"); return 1; }
                live.emplace_back(off, len);
                used += len;
            } else {
                const size_t k = rng() % live.size();
                if (!p.release(live[k].first)) { std::puts("FAIL release"); return 1; }
                used -= live[k].second;
                live.erase(live.begin() + k);
            }
            if (p.in_use() != used) { std::puts("FAIL accounting"); return 1; }
        }
        if (p.release(-256)) { std::puts("FAIL bogus release"); return 1; }
        for (auto &b : live) p.release(b.first);
        if (p.in_use() != 0 || p.n_free_blocks() != 1 || p.largest_free() != p.size()) {
            std::puts("FAIL coalesce"); return 1;
        }
    }
    std::puts("OK");
    return 0;
}
'''


def test_pool_allocator(tmp_path):
    csrc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2609_31258_amd", "csrc")
    src = tmp_path / "pool_test.cpp"
    src.write_text(HARNESS)
    exe = tmp_path / "pool_test"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Xlinker", "--no-as-needed", "-fsanitize=address,undefined",
                    "-I" + csrc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.strip()
    assert out == "OK"
