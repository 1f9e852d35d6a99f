"""Admission policy of the spectrum server (csrc/scheduler.h), exercised on the host.

The header is plain C++; a small driver is compiled with g++ and replays request
sequences against it.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1802_02854_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <string>
#include "scheduler.h"
using ftk::Admission;

static int failures = 0;
#define EXPECT(c) do { if (!(c)) { std::printf("FAIL line %d: %s\n", __LINE__, #c); ++failures; } } while (0)

static bool pick(Admission &a, uint64_t want)
{
    uint64_t t = 0; size_t b = 0;
    if (!a.pick(&t, &b)) return want == 0;
    return t == want;
}

int main()
{
    {   // FIFO within the budget and the worker limit
        Admission a(100, 2, 4);
        EXPECT(a.submit(1, 40)); EXPECT(a.submit(2, 40)); EXPECT(a.submit(3, 40));
        EXPECT(pick(a, 1)); EXPECT(pick(a, 2));
        EXPECT(pick(a, 0));                 // two running: worker limit
        EXPECT(a.in_use() == 80 && a.running() == 2);
        a.release(40);                      // a worker and 60 bytes free
        EXPECT(pick(a, 3));
        EXPECT(a.in_use() == 80 && a.peak() == 80);
    }
    {   // larger than the budget: refused
        Admission a(100, 4, 4);
        EXPECT(!a.submit(1, 101));
        EXPECT(a.submit(2, 100));
        EXPECT(pick(a, 2));
    }
    {   // backfill around a head that does not fit, at most max_bypass times
        Admission a(100, 8, 2);
        a.submit(1, 70); EXPECT(pick(a, 1));          // 30 left
        a.submit(2, 50);                              // head, does not fit
        a.submit(3, 10); a.submit(4, 10); a.submit(5, 10);
        EXPECT(pick(a, 3)); EXPECT(pick(a, 4));       // two bypasses
        EXPECT(pick(a, 0));                           // head is now protected
        a.release(70);                                // 80 left -> 20 in use
        EXPECT(pick(a, 2)); EXPECT(pick(a, 5));
        EXPECT(a.in_use() == 80 && a.waiting() == 0);
        EXPECT(a.peak() == 90);
    }
    {   // cancel
        Admission a(100, 1, 4);
        a.submit(1, 10); a.submit(2, 10);
        EXPECT(a.cancel(2)); EXPECT(!a.cancel(2));
        EXPECT(pick(a, 1)); EXPECT(a.waiting() == 0);
    }
    {   // never above the budget over a long random-ish stream
        Admission a(1000, 4, 4);
        uint64_t next = 1, x = 12345;
        size_t running_bytes[64]; uint64_t running_id[64]; int nr = 0;
        for (int step = 0; step < 20000; ++step) {
            x = x * 6364136223846793005ull + 1442695040888963407ull;
            const int op = (int)(x >> 62);
            if (op < 2) { a.submit(next++, 1 + (x >> 20) % 600); }
            else if (op == 2 && nr) { int i = (int)((x >> 30) % nr); a.release(running_bytes[i]);
                                      running_bytes[i] = running_bytes[nr - 1]; running_id[i] = running_id[nr - 1]; --nr; }
            else { uint64_t t; size_t b; if (a.pick(&t, &b)) { running_bytes[nr] = b; running_id[nr] = t; ++nr; } }
            EXPECT(a.in_use() <= a.budget());
            EXPECT(a.running() == nr && nr <= 4);
            if (failures) break;
        }
    }
    std::printf(failures ? "FAILED\n" : "OK\n");
    return failures ? 1 : 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_admission_policy(tmp_path):
    src = tmp_path / "drv.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "drv"
    # host-only driver: built with the address and undefined-behaviour sanitizers
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-Wall", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip().endswith("OK")
