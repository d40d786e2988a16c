"""The batched plan's autotuner cache file (csrc/tune_cache.cpp, host code),
compiled with AddressSanitizer and UndefinedBehaviorSanitizer into a small
driver: the last valid entry of a key wins, lines that do not parse (garbage,
truncated writes, values other than 1, 2 or 4, lines longer than any entry)
are skipped without hiding the lines after them, a missing file or an unset
path gives no choice, and stored entries are read back."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2202_10647_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1")

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include "tune_cache.hpp"
int main(int argc, char **argv)
{
    if (argc >= 4 && !std::strcmp(argv[1], "lookup")) {
        std::printf("%d\n", adk::tune_cache_lookup(std::strcmp(argv[2], "-") ? argv[2] : nullptr, argv[3]));
        return 0;
    }
    if (argc >= 5 && !std::strcmp(argv[1], "store")) {
        adk::tune_cache_store(argv[2], argv[3], std::atoi(argv[4]));
        return 0;
    }
    return 2;
}
"""

KEY = "gfx950|n=16777216|prec=1|wmax=6|b=0123456789abcdef"
OTHER = "gfx950|n=16777216|prec=1|wmax=1|b=fedcba9876543210"


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("tunecache")
    src = d / "driver.cpp"
    src.write_text(DRIVER)
    exe = d / "driver"
    subprocess.run(["g++", "-std=c++17", *SAN, "-I", CSRC, str(src), os.path.join(CSRC, "tune_cache.cpp"), "-o",
                    str(exe)], check=True, capture_output=True)
    return str(exe)


def lookup(driver, path, key=KEY):
    r = subprocess.run([driver, "lookup", str(path), key], capture_output=True, text=True, env=ENV)
    assert r.returncode == 0, r.stderr
    return int(r.stdout)


def test_missing_file_and_unset_path(driver, tmp_path):
    assert lookup(driver, tmp_path / "absent") == 0
    assert lookup(driver, "-") == 0


def test_store_then_lookup_last_entry_wins(driver, tmp_path):
    f = tmp_path / "cache"
    for cpl in (2, 4):
        subprocess.run([driver, "store", str(f), KEY, str(cpl)], check=True, env=ENV)
    subprocess.run([driver, "store", str(f), OTHER, "1"], check=True, env=ENV)
    assert f.read_text().splitlines() == [f"{KEY} 2", f"{KEY} 4", f"{OTHER} 1"]
    assert lookup(driver, f) == 4
    assert lookup(driver, f, OTHER) == 1
    assert lookup(driver, f, KEY + "x") == 0


def test_corrupt_lines_are_skipped(driver, tmp_path):
    f = tmp_path / "cache"
    f.write_text("\n".join([
        "garbage without a value",
        f"{KEY} 3",             # not a cells-per-lane choice
        f"{KEY} 4x",            # trailing junk
        f"{KEY}",               # value missing
        "x" * 5000,             # longer than any entry
        f"{KEY} 2",             # valid, after all of the above
        f"{KEY[:20]}",          # a truncated write at the end
    ]))
    assert lookup(driver, f) == 2
    f.write_text("\x00\xff binary junk\n" + f"{OTHER} 4\n")
    assert lookup(driver, f, OTHER) == 4
    assert lookup(driver, f) == 0


def test_only_invalid_entries_means_retune(driver, tmp_path):
    f = tmp_path / "cache"
    f.write_text(f"{KEY} 0\n{KEY} -1\n{KEY} 8\n{KEY} two\n")
    assert lookup(driver, f) == 0
