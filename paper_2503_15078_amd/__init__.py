"""MI355X-native local-global hyperelastic solver with frictional contact (HIP, gfx950)."""
