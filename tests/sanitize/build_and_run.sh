#!/bin/bash
# Build the library's sources with AddressSanitizer and
# UndefinedBehaviorSanitizer (each -fsanitize= after -Xarch_host, so no
# device code is built with them) and run host_calls.cpp against them.
# Usage: tests/sanitize/build_and_run.sh <build directory>
set -e
HERE=$(cd "$(dirname "$0")" && pwd)
SRC=$HERE/../../paper_1705_03838_amd/csrc
OUT=${1:-/tmp/opf_sanitize}
mkdir -p "$OUT"
FLAGS="-O1 -g -std=c++17 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-sanitize-recover=all -w"
pids=()
for f in opf_host opf_transform opf_solve opf_factor opf_mlp; do
  /opt/rocm/bin/hipcc $FLAGS -c "$SRC/$f.hip" -o "$OUT/$f.o" & pids+=($!)
done
for p in "${pids[@]}"; do wait $p; done
/opt/rocm/lib/llvm/bin/clang++ -O1 -g -std=c++17 -fsanitize=address,undefined -fno-sanitize-recover=all \
  -c "$HERE/host_calls.cpp" -o "$OUT/host_calls.o"
/opt/rocm/bin/hipcc --offload-arch=gfx950 -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined \
  "$OUT/host_calls.o" "$OUT"/opf_*.o -o "$OUT/host_calls"
ASAN_OPTIONS=detect_leaks=1 UBSAN_OPTIONS=print_stacktrace=1 "$OUT/host_calls" "$OUT"
