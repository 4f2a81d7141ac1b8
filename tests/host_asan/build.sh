#!/bin/bash
# Builds the C-ABI library with AddressSanitizer on its host code only (device
# code is compiled as in the product build) and the asan_driver harness.
# Output: tests/host_asan/_build/asan_driver. Run it with
#   ASAN_OPTIONS=detect_leaks=0:verify_asan_link_order=0 tests/host_asan/_build/asan_driver
set -e
HERE=$(cd "$(dirname "$0")" && pwd)
ROOT=$(cd "$HERE/../.." && pwd)
OUT=$HERE/_build
mkdir -p "$OUT"
HIPCC=${HIPCC:-/opt/rocm/bin/hipcc}
FLAGS="-O1 -g -fPIC -std=c++17 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops -Xarch_host -fsanitize=address -Xarch_host -fno-omit-frame-pointer -I$ROOT/include -I$ROOT/paper_1009_3308_amd/csrc"
SRCS="host_numerics.cpp nse_api.cpp legendre_table.hip synthesis.hip ring_fft.hip analysis.hip contract_lp.hip adjoint.hip ensemble.hip ndf_adaptive.hip diagnostics.hip"
pids=""
for f in $SRCS; do
  "$HIPCC" -x hip $FLAGS -c "$ROOT/paper_1009_3308_amd/csrc/$f" -o "$OUT/${f%.*}.o" &
  pids="$pids $!"
done
for p in $pids; do wait $p; done
"$HIPCC" -x hip $FLAGS -c "$HERE/asan_driver.cpp" -o "$OUT/asan_driver.o"
"$HIPCC" --offload-arch=gfx950 -Xarch_host -fsanitize=address "$OUT"/*.o -o "$OUT/asan_driver"
echo "built $OUT/asan_driver"
