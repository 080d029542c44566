#!/bin/bash
# Builds host_sanitize_driver: the library's sources and the driver with
# AddressSanitizer and UndefinedBehaviorSanitizer on the host code only (every
# -fsanitize follows -Xarch_host; device code is not instrumented), linked
# into one executable so that the sanitizer runtime comes with it.
# Usage: tests/sanitize/build.sh [output directory]   (default: tests/sanitize/_build)
# SANITIZE (default "address undefined") lists the sanitizers; empty builds
# the same executable without any.
set -e
HERE="$(cd "$(dirname "$0")" && pwd)"
ROOT="$(cd "$HERE/../.." && pwd)"
OUT="${1:-$HERE/_build}"
mkdir -p "$OUT"
SAN=()
for s in ${SANITIZE-address undefined}; do
  SAN+=(-Xarch_host "-fsanitize=$s")
done
FLAGS=(--offload-arch=gfx950 -O3 -std=c++17 -Xarch_host -g
       -Xclang -target-feature -Xclang -packed-fp32-ops
       -mllvm -amdgpu-mfma-vgpr-form=1 -Wno-unused-result
       "${SAN[@]}" -Xarch_host -fno-omit-frame-pointer -Xarch_host -fno-sanitize-recover=undefined)
OBJS=()
for src in "$ROOT"/paper_2006_15234_amd/csrc/*.hip; do
  OBJS+=("$OUT/$(basename "${src%.hip}").o")
done
export OUT ROOT
export FLAGS_STR="${FLAGS[*]}"
# at most six compilers at once (memory)
ls "$ROOT"/paper_2006_15234_amd/csrc/*.hip | xargs -P 6 -I{} bash -c \
  'src="{}"; hipcc $FLAGS_STR -I"$ROOT/include" -c "$src" -o "$OUT/$(basename "${src%.hip}").o"'
hipcc "${FLAGS[@]}" -I"$ROOT/include" -x hip -c "$HERE/host_sanitize_driver.cpp" -o "$OUT/driver.o"
hipcc --offload-arch=gfx950 "${SAN[@]}" "$OUT/driver.o" "${OBJS[@]}" -o "$OUT/host_sanitize_driver"
rm -f "$OUT"/*.o
echo "built $OUT/host_sanitize_driver"
